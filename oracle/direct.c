/* Direct FP64 sums of the FIRM operators at selected outputs (test infrastructure only).
 *
 * Plain C, no approximation: every output is the full sum over all images m and
 * all disk points k of its defining equation.  The only rewriting is
 *   exp(i <n, xi_{k,m}>) = exp(i (2 pi/N) k1 <n, c1_m>) * exp(i (2 pi/N) k2 <n, c2_m>),
 * with c1_m, c2_m the first two columns of R_m^{-1}, which is the definition of
 * xi_{k,m} = R_m^{-1}(omega_k1, omega_k2, 0) (eq. forward-projector) written per
 * factor; each factor is evaluated with cos/sin, never by recurrence.
 *
 * Layouts: rotations M x 9 row-major; CTF table G x (N*N/4 + 1) indexed by
 * q = k1^2 + k2^2 (group g per image, NULL table means h = 1); slices M x P
 * complex interleaved (re, im) in the canonical disk order (k1 ascending, then
 * k2 ascending, ||k|| <= N/2); shifts M x 2 (NULL = none).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static const double TWO_PI = 6.283185307179586476925286766559;

/* columns 1 and 2 of the inverse of a 3x3 matrix (adjugate / determinant) */
static void inverse_cols12(const double* R, double c1[3], double c2[3]) {
    double a = R[0], b = R[1], c = R[2], d = R[3], e = R[4], f = R[5], g = R[6], h = R[7], i = R[8];
    double A = e * i - f * h, B = -(d * i - f * g), C = d * h - e * g;
    double det = a * A + b * B + c * C;
    /* inverse = adj / det; adj(j,k) = cofactor(k,j) */
    double inv[9];
    inv[0] = A / det;               inv[1] = -(b * i - c * h) / det; inv[2] = (b * f - c * e) / det;
    inv[3] = B / det;               inv[4] = (a * i - c * g) / det;  inv[5] = -(a * f - c * d) / det;
    inv[6] = C / det;               inv[7] = -(a * h - b * g) / det; inv[8] = (a * e - b * d) / det;
    c1[0] = inv[0]; c1[1] = inv[3]; c1[2] = inv[6];
    c2[0] = inv[1]; c2[1] = inv[4]; c2[2] = inv[7];
}

static int64_t disk_rows(int N, int* k1s, int* k2lo, int* k2hi, int64_t* rowoff) {
    int64_t P = 0;
    int rows = 0;
    for (int k1 = -N / 2; k1 <= N / 2; ++k1) {
        int lo = 1, hi = 0;
        for (int k2 = -N / 2; k2 <= N / 2; ++k2)
            if (4 * (k1 * k1 + k2 * k2) <= N * N) { if (lo > hi) lo = k2; hi = k2; }
        k1s[rows] = k1; k2lo[rows] = lo; k2hi[rows] = hi; rowoff[rows] = P;
        P += (hi >= lo) ? (hi - lo + 1) : 0;
        ++rows;
    }
    return P;
}

int64_t oracle_slice_points(int N) {
    int k1s[1030], lo[1030], hi[1030];
    int64_t off[1030];
    return disk_rows(N, k1s, lo, hi, off);
}

/* weight of image m at q: h or h^2 */
static inline double ctf_h(const float* table, const int32_t* group, int Q, int m, int q) {
    if (!table) return 1.0;
    int g = group ? group[m] : 0;
    return (double)table[(int64_t)g * Q + q];
}

/* Ker(n) = sum_m sum_k exp(i <n, xi>) h_m^2  (eq. kernel), at K offsets; out K x 2 (re, im). */
void oracle_kernel_at(int N, int M, const double* rot, const int32_t* group, const float* table,
                      int K, const int32_t* offs, double* out, int nthreads) {
    int k1s[1030], lo[1030], hi[1030];
    int64_t off[1030];
    disk_rows(N, k1s, lo, hi, off);
    int rows = N + 1, Q = N * N / 4 + 1;
    for (int t = 0; t < K; ++t) {
        double n[3] = {offs[3 * t], offs[3 * t + 1], offs[3 * t + 2]};
        double sre = 0.0, sim = 0.0;
#pragma omp parallel for reduction(+ : sre, sim) schedule(static) num_threads(nthreads)
        for (int m = 0; m < M; ++m) {
            double c1[3], c2[3];
            inverse_cols12(rot + 9 * (int64_t)m, c1, c2);
            double u = n[0] * c1[0] + n[1] * c1[1] + n[2] * c1[2];
            double v = n[0] * c2[0] + n[1] * c2[1] + n[2] * c2[2];
            double e2r[1030], e2i[1030];
            for (int k2 = -N / 2; k2 <= N / 2; ++k2) {
                double a = TWO_PI * k2 * v / N;
                e2r[k2 + N / 2] = cos(a); e2i[k2 + N / 2] = sin(a);
            }
            double mr = 0.0, mi = 0.0;
            for (int r = 0; r < rows; ++r) {
                int k1 = k1s[r];
                double a = TWO_PI * k1 * u / N, e1r = cos(a), e1i = sin(a);
                for (int k2 = lo[r]; k2 <= hi[r]; ++k2) {
                    double hh = ctf_h(table, group, Q, m, k1 * k1 + k2 * k2);
                    double w = hh * hh;
                    double pr = e1r * e2r[k2 + N / 2] - e1i * e2i[k2 + N / 2];
                    double pi = e1r * e2i[k2 + N / 2] + e1i * e2r[k2 + N / 2];
                    mr += w * pr; mi += w * pi;
                }
            }
            sre += mr; sim += mi;
        }
        out[2 * t] = sre; out[2 * t + 1] = sim;
    }
}

/* (A* g)(n) = sum_m sum_k exp(i <n, xi>) h_m g_{k,m}  (eq. backprojection), with g the
 * re-centred slices b(k,m) exp(+i <omega_k, s_m>); at K voxel offsets n; out K x 2. */
void oracle_backproject_at(int N, int M, const double* rot, const int32_t* group, const float* table,
                           const double* shifts, const float* b, int K, const int32_t* vox,
                           double* out, int nthreads) {
    int k1s[1030], lo[1030], hi[1030];
    int64_t off[1030];
    int64_t P = disk_rows(N, k1s, lo, hi, off);
    int rows = N + 1, Q = N * N / 4 + 1;
    for (int t = 0; t < K; ++t) {
        double n[3] = {vox[3 * t], vox[3 * t + 1], vox[3 * t + 2]};
        double sre = 0.0, sim = 0.0;
#pragma omp parallel for reduction(+ : sre, sim) schedule(static) num_threads(nthreads)
        for (int m = 0; m < M; ++m) {
            double c1[3], c2[3];
            inverse_cols12(rot + 9 * (int64_t)m, c1, c2);
            double u = n[0] * c1[0] + n[1] * c1[1] + n[2] * c1[2];
            double v = n[0] * c2[0] + n[1] * c2[1] + n[2] * c2[2];
            double s1 = shifts ? shifts[2 * (int64_t)m] : 0.0, s2 = shifts ? shifts[2 * (int64_t)m + 1] : 0.0;
            double mr = 0.0, mi = 0.0;
            for (int r = 0; r < rows; ++r) {
                int k1 = k1s[r];
                for (int k2 = lo[r]; k2 <= hi[r]; ++k2) {
                    int64_t j = (int64_t)m * P + off[r] + (k2 - lo[r]);
                    double gr = b[2 * j], gi = b[2 * j + 1];
                    /* re-centring phase exp(+i <omega, s>) and the back-projection phase */
                    double ph = TWO_PI * (k1 * s1 + k2 * s2) / N + TWO_PI * (k1 * u + k2 * v) / N;
                    double cr = cos(ph), ci = sin(ph);
                    double hh = ctf_h(table, group, Q, m, k1 * k1 + k2 * k2);
                    mr += hh * (cr * gr - ci * gi);
                    mi += hh * (cr * gi + ci * gr);
                }
            }
            sre += mr; sim += mi;
        }
        out[2 * t] = sre; out[2 * t + 1] = sim;
    }
}

/* Clean slices of a Gaussian-blob volume, closed form (projection-slice theorem,
 * eq. continuous_fps): b(k,m) = h exp(-i <omega_k, s_m>) sum_b a_b (2 pi s_b^2)^{3/2}
 * exp(-s_b^2 ||xi||^2 / 2) exp(-i <c_b, xi>); s_b = 0 is a point source of weight a_b.
 * out M x P complex interleaved (float64). */
void oracle_blob_slices(int N, int M, const double* rot, const int32_t* group, const float* table,
                        const double* shifts, int B, const double* centers, const double* sigmas,
                        const double* amps, double* out, int nthreads) {
    int k1s[1030], lo[1030], hi[1030];
    int64_t off[1030];
    int64_t P = disk_rows(N, k1s, lo, hi, off);
    int rows = N + 1, Q = N * N / 4 + 1;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
    for (int m = 0; m < M; ++m) {
        double c1[3], c2[3];
        inverse_cols12(rot + 9 * (int64_t)m, c1, c2);
        double s1 = shifts ? shifts[2 * (int64_t)m] : 0.0, s2 = shifts ? shifts[2 * (int64_t)m + 1] : 0.0;
        for (int r = 0; r < rows; ++r) {
            int k1 = k1s[r];
            for (int k2 = lo[r]; k2 <= hi[r]; ++k2) {
                double w1 = TWO_PI * k1 / N, w2 = TWO_PI * k2 / N;
                double xi[3] = {w1 * c1[0] + w2 * c2[0], w1 * c1[1] + w2 * c2[1], w1 * c1[2] + w2 * c2[2]};
                double x2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
                double re = 0.0, im = 0.0;
                for (int bb = 0; bb < B; ++bb) {
                    double s = sigmas[bb];
                    double amp = s > 0 ? amps[bb] * pow(TWO_PI * s * s, 1.5) * exp(-0.5 * s * s * x2) : amps[bb];
                    double ph = -(centers[3 * bb] * xi[0] + centers[3 * bb + 1] * xi[1] + centers[3 * bb + 2] * xi[2]);
                    re += amp * cos(ph); im += amp * sin(ph);
                }
                double hh = ctf_h(table, group, Q, m, k1 * k1 + k2 * k2);
                double sp = -(w1 * s1 + w2 * s2);
                double cr = cos(sp), ci = sin(sp);
                int64_t j = (int64_t)m * P + off[r] + (k2 - lo[r]);
                out[2 * j] = hh * (cr * re - ci * im);
                out[2 * j + 1] = hh * (cr * im + ci * re);
            }
        }
    }
}
