/*
 * CPU oracle for Fock-state amplitudes through beam-splitter circuits.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table
 * or constant with the GPU path.
 *
 * What it computes is the plain definition of the quantity the path sum
 * reaches (Sec. II and the Appendix of the paper):
 *
 *   <T| U_P |S> = Per(U[T,S]) / sqrt(prod_i s_i! * prod_j t_j!)
 *
 * where U is the M x M matrix that maps input creation operators to output
 * creation operators (rows = output modes, columns = input modes), U is the
 * product of the embedded 2x2 beam-splitter matrices in application order
 * (the first beam splitter acts first, so it is the right-most factor), and
 * U[T,S] repeats output row j t_j times and input column i s_i times.
 *
 * Precision: matrix composition and the Ryser sum are accumulated in
 * long double (x87 80-bit); inputs and outputs are double.  Each permanent
 * also returns an a-posteriori bound on its own rounding error.
 *
 * Functions:
 *   orc_permanent_ryser  Ryser's formula, Gray-code subset order
 *   orc_permanent_brute  sum over all permutations (definition; tiny n)
 *   orc_bs_amplitude     Appendix: single-BS amplitude as the permanent of the
 *                        repeated 2x2 matrix divided by sqrt(x1!x2!y1!y2!)
 *   orc_fock_amplitude   the definition for an arbitrary matrix
 *   orc_compose          U = L_K ... L_1
 *   orc_amplitude(s)     the definition above, one pattern / a batch
 *   orc_pathsum          Eq. (1): explicit sum over every sequence of
 *                        intermediate Fock configurations (no pruning beyond
 *                        photon-number conservation); tiny inputs only
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double ld;
typedef struct { ld re, im; } lcx;

static lcx cx(ld re, ld im) { lcx z; z.re = re; z.im = im; return z; }
static lcx cadd(lcx a, lcx b) { return cx(a.re + b.re, a.im + b.im); }
static lcx csub(lcx a, lcx b) { return cx(a.re - b.re, a.im - b.im); }
static lcx cmul(lcx a, lcx b) { return cx(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
static ld cabs_l(lcx a) { return sqrtl(a.re * a.re + a.im * a.im); }

/* Eq. (bs_matrix): [[cos t, -e^{-i p} sin t], [e^{i p} sin t, cos t]],
 * B[0] = U11, B[1] = U12, B[2] = U21, B[3] = U22 with row = output mode,
 * column = input mode (1 = upper). */
static void bs_matrix_l(double theta, double phi, lcx B[4])
{
    ld c = cosl((ld)theta), s = sinl((ld)theta);
    ld cp = cosl((ld)phi), sp = sinl((ld)phi);
    B[0] = cx(c, 0);
    B[1] = cx(-cp * s, sp * s);
    B[2] = cx(cp * s, sp * s);
    B[3] = cx(c, 0);
}

/* Ryser: Per(A) = (-1)^n sum_{X subset of columns} (-1)^{|X|} prod_i sum_{j in X} a_ij,
 * visiting subsets in Gray-code order so each step adds or removes one column.
 * err_bound receives (n+3) * 2^-63 * sum_X |prod_i rowsum_i(X)|, a bound on the
 * accumulated rounding error of the long-double evaluation. */
static lcx ryser_l(int n, const lcx *a, ld *absum)
{
    if (n == 0) { if (absum) *absum = 1; return cx(1, 0); }
    lcx rs[64];
    for (int i = 0; i < n; i++) rs[i] = cx(0, 0);
    lcx total = cx(0, 0);
    ld mag = 0;
    uint64_t ns = (uint64_t)1 << n;
    uint64_t gray_prev = 0;
    for (uint64_t k = 1; k < ns; k++) {
        uint64_t g = k ^ (k >> 1);
        uint64_t diff = g ^ gray_prev;
        int j = __builtin_ctzll(diff);
        int add = (g >> j) & 1;
        for (int i = 0; i < n; i++)
            rs[i] = add ? cadd(rs[i], a[i * n + j]) : csub(rs[i], a[i * n + j]);
        lcx p = rs[0];
        for (int i = 1; i < n; i++) p = cmul(p, rs[i]);
        int pop = __builtin_popcountll(g);
        if ((pop & 1) == (n & 1)) total = cadd(total, p);   /* (-1)^{n+|X|} = +1 */
        else total = csub(total, p);
        mag += cabs_l(p);
        gray_prev = g;
    }
    if (absum) *absum = mag;
    return total;
}

int orc_permanent_ryser(int n, const double *a, double *out, double *err_bound)
{
    if (n < 0 || n > 40) return 1;
    lcx *al = (lcx *)malloc(sizeof(lcx) * (size_t)(n > 0 ? n * n : 1));
    for (int i = 0; i < n * n; i++) al[i] = cx(a[2 * i], a[2 * i + 1]);
    ld mag;
    lcx p = ryser_l(n, al, &mag);
    free(al);
    out[0] = (double)p.re; out[1] = (double)p.im;
    if (err_bound) *err_bound = (double)((ld)(n + 3) * ldexpl(1.0L, -63) * mag);
    return 0;
}

/* Definition: sum over all permutations sigma of prod_i a_{i,sigma(i)}. */
static lcx brute_rec(int n, const lcx *a, int row, uint64_t used, lcx acc)
{
    if (row == n) return acc;
    lcx s = cx(0, 0);
    for (int j = 0; j < n; j++) {
        if (used & ((uint64_t)1 << j)) continue;
        s = cadd(s, brute_rec(n, a, row + 1, used | ((uint64_t)1 << j), cmul(acc, a[row * n + j])));
    }
    return s;
}

int orc_permanent_brute(int n, const double *a, double *out)
{
    if (n < 0 || n > 10) return 1;
    lcx al[100];
    for (int i = 0; i < n * n; i++) al[i] = cx(a[2 * i], a[2 * i + 1]);
    lcx p = brute_rec(n, al, 0, 0, cx(1, 0));
    out[0] = (double)p.re; out[1] = (double)p.im;
    return 0;
}

static ld lfact(int k) { ld f = 1; for (int i = 2; i <= k; i++) f *= i; return f; }

/* Amplitude of the sub-matrix of Umat (m x m, rows = outputs) selected by
 * repeating output row j T[j] times and input column i S[i] times. */
static lcx amp_from_matrix(int m, const lcx *Umat, const int *S, const int *T, ld *errb)
{
    int nS = 0, nT = 0;
    for (int i = 0; i < m; i++) { nS += S[i]; nT += T[i]; }
    if (nS != nT) { if (errb) *errb = 0; return cx(0, 0); }
    int n = nS;
    int rows[64], cols[64];
    int k = 0;
    for (int j = 0; j < m; j++) for (int r = 0; r < T[j]; r++) rows[k++] = j;
    k = 0;
    for (int i = 0; i < m; i++) for (int r = 0; r < S[i]; r++) cols[k++] = i;
    lcx *sub = (lcx *)malloc(sizeof(lcx) * (size_t)(n > 0 ? n * n : 1));
    for (int r = 0; r < n; r++)
        for (int c = 0; c < n; c++) sub[r * n + c] = Umat[rows[r] * m + cols[c]];
    ld mag;
    lcx per = ryser_l(n, sub, &mag);
    free(sub);
    ld norm = 1;
    for (int i = 0; i < m; i++) norm *= lfact(S[i]) * lfact(T[i]);
    norm = sqrtl(norm);
    if (errb) *errb = (ld)(n + 3) * ldexpl(1.0L, -63) * mag / norm;
    return cx(per.re / norm, per.im / norm);
}

/* Appendix: <y1,y2|BS|x1,x2> as the permanent of the 2x2 matrix with output
 * row 1 repeated y1 times, row 2 y2 times, input column 1 x1 times, column 2
 * x2 times, over sqrt(x1!x2!y1!y2!).  Zero unless x1+x2 = y1+y2. */
int orc_bs_amplitude(double theta, double phi, int x1, int x2, int y1, int y2, double *out)
{
    if (x1 < 0 || x2 < 0 || y1 < 0 || y2 < 0 || x1 + x2 > 40) return 1;
    lcx B[4];
    bs_matrix_l(theta, phi, B);
    int S[2] = {x1, x2}, T[2] = {y1, y2};
    lcx a = amp_from_matrix(2, B, S, T, NULL);
    out[0] = (double)a.re; out[1] = (double)a.im;
    return 0;
}

/* Same definition for an arbitrary m x m matrix (row-major, re/im
 * interleaved, rows = outputs): Per(U[T,S]) / sqrt(prod s! prod t!). */
int orc_fock_amplitude(int m, const double *Umat, const int *S, const int *T, double *out)
{
    if (m < 1 || m > 64) return 1;
    int n = 0;
    for (int i = 0; i < m; i++) { if (S[i] < 0 || T[i] < 0) return 1; n += S[i]; }
    if (n > 40) return 1;
    lcx *U = (lcx *)malloc(sizeof(lcx) * (size_t)m * m);
    for (int i = 0; i < m * m; i++) U[i] = cx(Umat[2 * i], Umat[2 * i + 1]);
    lcx a = amp_from_matrix(m, U, S, T, NULL);
    free(U);
    out[0] = (double)a.re; out[1] = (double)a.im;
    return 0;
}

/* U = L_K ... L_1 for beam splitters given in application order.
 * Umat_out: m*m complex (re,im interleaved), row-major, rows = outputs. */
static int compose_l(int m, int nbs, const int *ma, const int *mb, const double *theta,
                     const double *phi, lcx *U)
{
    for (int r = 0; r < m; r++)
        for (int c = 0; c < m; c++) U[r * m + c] = cx(r == c ? 1 : 0, 0);
    for (int g = 0; g < nbs; g++) {
        int a = ma[g], b = mb[g];
        if (a < 0 || b < 0 || a >= m || b >= m || a == b) return 1;
        lcx B[4];
        bs_matrix_l(theta[g], phi[g], B);
        for (int c = 0; c < m; c++) {
            lcx ua = U[a * m + c], ub = U[b * m + c];
            U[a * m + c] = cadd(cmul(B[0], ua), cmul(B[1], ub));
            U[b * m + c] = cadd(cmul(B[2], ua), cmul(B[3], ub));
        }
    }
    return 0;
}

int orc_compose(int m, int nbs, const int *ma, const int *mb, const double *theta,
                const double *phi, double *Uout)
{
    if (m < 1 || m > 256) return 1;
    lcx *U = (lcx *)malloc(sizeof(lcx) * (size_t)m * m);
    int rc = compose_l(m, nbs, ma, mb, theta, phi, U);
    if (!rc)
        for (int i = 0; i < m * m; i++) { Uout[2 * i] = (double)U[i].re; Uout[2 * i + 1] = (double)U[i].im; }
    free(U);
    return rc;
}

int orc_amplitude(int m, const int *S, const int *T, int nbs, const int *ma, const int *mb,
                  const double *theta, const double *phi, double *out, double *err_bound)
{
    if (m < 1 || m > 64) return 1;
    int n = 0;
    for (int i = 0; i < m; i++) { if (S[i] < 0 || T[i] < 0) return 1; n += S[i]; }
    if (n > 40) return 1;
    lcx *U = (lcx *)malloc(sizeof(lcx) * (size_t)m * m);
    if (compose_l(m, nbs, ma, mb, theta, phi, U)) { free(U); return 1; }
    ld eb;
    lcx a = amp_from_matrix(m, U, S, T, &eb);
    free(U);
    out[0] = (double)a.re; out[1] = (double)a.im;
    if (err_bound) *err_bound = (double)eb;
    return 0;
}

/* Batch form: one S, nT output patterns (row-major nT x m).  Parallel over
 * patterns with OpenMP when nthreads > 1.  Returns the thread count used in
 * *threads_used. */
int orc_amplitudes(int m, const int *S, int nT, const int *T, int nbs, const int *ma,
                   const int *mb, const double *theta, const double *phi, double *out,
                   double *err_bound, int nthreads, int *threads_used)
{
    if (m < 1 || m > 64 || nT < 0) return 1;
    for (int i = 0; i < m; i++) if (S[i] < 0) return 1;
    lcx *U = (lcx *)malloc(sizeof(lcx) * (size_t)m * m);
    if (compose_l(m, nbs, ma, mb, theta, phi, U)) { free(U); return 1; }
    int used = 1;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
    #pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int p = 0; p < nT; p++) {
        ld eb;
        lcx a = amp_from_matrix(m, U, S, T + (size_t)p * m, &eb);
        out[2 * p] = (double)a.re; out[2 * p + 1] = (double)a.im;
        if (err_bound) err_bound[p] = (double)eb;
    }
#ifdef _OPENMP
    used = nthreads;
#endif
    if (threads_used) *threads_used = used;
    free(U);
    return 0;
}

/* Eq. (1), written out: depth-first over every beam splitter in application
 * order, each BS taking every output split (y1, N - y1) of its N input
 * photons; a path is a full sequence of such choices, its weight is the
 * product of the single-BS amplitudes (orc_bs_amplitude), and the paths
 * whose final configuration equals T are summed.  No light-cone pruning: this
 * is exponential and meant for tiny circuits.  *npaths counts the valid
 * paths (those ending in T), including ones whose weight is numerically 0. */
typedef struct {
    int m, nbs;
    const int *ma, *mb;
    const double *theta, *phi;
    const int *T;
    lcx acc;
    double npaths;
} pathsum_ctx;

static void pathsum_rec(pathsum_ctx *cx_, int g, int *occ, lcx w)
{
    if (g == cx_->nbs) {
        for (int i = 0; i < cx_->m; i++) if (occ[i] != cx_->T[i]) return;
        cx_->acc = cadd(cx_->acc, w);
        cx_->npaths += 1;
        return;
    }
    int a = cx_->ma[g], b = cx_->mb[g];
    int x1 = occ[a], x2 = occ[b], N = x1 + x2;
    lcx B[4];
    bs_matrix_l(cx_->theta[g], cx_->phi[g], B);
    for (int y1 = 0; y1 <= N; y1++) {
        int S2[2] = {x1, x2}, T2[2] = {y1, N - y1};
        lcx f = amp_from_matrix(2, B, S2, T2, NULL);
        occ[a] = y1; occ[b] = N - y1;
        pathsum_rec(cx_, g + 1, occ, cmul(w, f));
    }
    occ[a] = x1; occ[b] = x2;
}

int orc_pathsum(int m, const int *S, const int *T, int nbs, const int *ma, const int *mb,
                const double *theta, const double *phi, double *out, double *npaths)
{
    if (m < 1 || m > 64) return 1;
    int occ[64];
    int nS = 0, nT = 0;
    for (int i = 0; i < m; i++) { occ[i] = S[i]; nS += S[i]; nT += T[i]; }
    for (int g = 0; g < nbs; g++)
        if (ma[g] < 0 || mb[g] < 0 || ma[g] >= m || mb[g] >= m || ma[g] == mb[g]) return 1;
    pathsum_ctx c;
    c.m = m; c.nbs = nbs; c.ma = ma; c.mb = mb; c.theta = theta; c.phi = phi; c.T = T;
    c.acc = cx(0, 0); c.npaths = 0;
    if (nS == nT) pathsum_rec(&c, 0, occ, cx(1, 0));
    out[0] = (double)c.acc.re; out[1] = (double)c.acc.im;
    if (npaths) *npaths = c.npaths;
    return 0;
}
