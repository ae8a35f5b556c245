/*
 * CPU oracle for the bosonic multiconfigurational operators of
 * Andriati & Gammal, "Hashing algorithms, optimized mappings and massive
 * parallelization of multiconfigurational methods for bosons"
 * (arXiv:2005.13679).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code with the GPU library.
 *
 * Deliberately plain and slow:
 *   - N_c(n, m) comes from its binomial definition (small arguments from a
 *     table of the same values, filled once at load);
 *   - configuration -> index is the total particle cost of Eq. (TotalCost),
 *     one particle at a time;
 *   - index -> configuration bisects on that rank, orbital by orbital;
 *   - H.C and the density matrices are obtained by applying creation and
 *     annihilation operators to occupation vectors, one operator at a time,
 *     with no jump tables and no case table;
 *   - every reduction uses Neumaier-compensated summation.
 * Rows (or density-matrix elements) are distributed over OpenMP threads; each
 * thread owns its outputs, so results do not depend on the thread count.
 *
 * Complex arrays are interleaved (re, im) doubles.  h is h[k*M + l],
 * g is g[((k*M + s)*M + q)*M + l]; rho1 and rho2 use the same layouts.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_MAXM 64

/* ---------------------------------------------------------------------- */
/* Eq. (nc): N_c(n, m) = (n + m - 1)! / (n! (m - 1)!), with N_c(n, 0) = 0   */
/* (Eq. TotalCost).  Returns -1 if the value does not fit in int64.         */
/* ---------------------------------------------------------------------- */
static int64_t nc_definition(int64_t n, int64_t m)
{
    if (m <= 0 || n < 0) return 0;
    int64_t a = n + m - 1;          /* C(a, b) with b = m - 1 */
    int64_t b = m - 1;
    if (b > a - b) b = a - b;
    unsigned __int128 r = 1;
    for (int64_t i = 1; i <= b; ++i) {
        r = r * (unsigned __int128)(a - b + i) / (unsigned __int128)i;
        if (r > (unsigned __int128)INT64_MAX) return -1;
    }
    return (int64_t)r;
}

/* The hash below asks for N_c(i, m) once per particle, so small arguments
 * are answered from a table that nc_definition fills once when the library
 * is loaded; everything else is computed from the definition. */
#define ORC_NC_TAB_N 4096
#define ORC_NC_TAB_M 32
static int64_t nc_table[ORC_NC_TAB_M][ORC_NC_TAB_N];

__attribute__((constructor)) static void nc_table_fill(void)
{
    for (int64_t m = 0; m < ORC_NC_TAB_M; ++m)
        for (int64_t n = 0; n < ORC_NC_TAB_N; ++n)
            nc_table[m][n] = nc_definition(n, m);
}

int64_t orc_nc(int64_t n, int64_t m)
{
    if (n >= 0 && n < ORC_NC_TAB_N && m >= 0 && m < ORC_NC_TAB_M) return nc_table[m][n];
    return nc_definition(n, m);
}

/* Configuration -> index, written from Eq. (TotalCost): list the particles
 * by nondecreasing orbital, p_1 <= p_2 <= ... <= p_N; particle i (1-based)
 * costs N_c(i, p_i), and the index is the total cost.  Particles in orbital
 * 0 cost nothing (N_c(i, 0) = 0).  This is the same map Algorithm 1
 * computes, evaluated from the lowest orbital up and without a basket. */
int64_t orc_hash(int32_t N, int32_t M, const int32_t *n)
{
    (void)N;
    int64_t index = 0;
    int64_t i = 0;                          /* particles listed so far */
    for (int32_t orb = 0; orb < M; ++orb) {
        for (int32_t c = 0; c < n[orb]; ++c) {
            ++i;
            index += orc_nc(i, orb);
        }
    }
    return index;
}

/* Index -> configuration, by bisection on the rank of orc_hash.  The order
 * compares n_{M-1} first, then n_{M-2}, ... (orbital M-1 most significant).
 * With the orbitals above m already fixed and `left` particles still to
 * place, the first configuration with n_m = t puts the other left - t
 * particles into orbital 0, and its rank grows with t; so n_m is the largest
 * t whose first configuration does not rank above beta.  What is left after
 * orbital 1 goes to orbital 0.  Returns 0 on success, -1 if beta is outside
 * [0, N_c(N, M)). */
int orc_unhash(int32_t N, int32_t M, int64_t beta, int32_t *n)
{
    if (beta < 0 || beta >= orc_nc(N, M)) return -1;
    for (int32_t i = 0; i < M; ++i) n[i] = 0;
    int32_t left = N;
    for (int32_t m = M - 1; m >= 1; --m) {
        int32_t lo = 0, hi = left;          /* invariant: rank(lo) <= beta */
        while (lo < hi) {
            int32_t mid = lo + (hi - lo + 1) / 2;
            n[m] = mid;
            n[0] = left - mid;
            if (orc_hash(N, M, n) <= beta) lo = mid;
            else hi = mid - 1;
        }
        n[m] = lo;
        n[0] = 0;
        left -= lo;
    }
    n[0] = left;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Operator algebra on occupation vectors.                                  */
/* a_j |..n_j..>  = sqrt(n_j)   |..n_j - 1..>   (zero if n_j = 0)          */
/* a+_j|..n_j..>  = sqrt(n_j+1) |..n_j + 1..>                               */
/* The amplitude is returned as the product of the integers under the       */
/* square roots (exact in double for the sizes used), or 0 if the string    */
/* annihilates the state.                                                   */
/* ---------------------------------------------------------------------- */
static double annihilate(int32_t *n, int32_t j)
{
    if (n[j] == 0) return 0.0;
    double f = (double)n[j];
    n[j] -= 1;
    return f;
}

static double create(int32_t *n, int32_t j)
{
    n[j] += 1;
    return (double)n[j];
}

/* Neumaier compensated accumulator */
typedef struct { double sum, comp; } nsum;

static void nadd(nsum *a, double x)
{
    double t = a->sum + x;
    if (fabs(a->sum) >= fabs(x)) a->comp += (a->sum - t) + x;
    else                          a->comp += (x - t) + a->sum;
    a->sum = t;
}

static double nval(const nsum *a) { return a->sum + a->comp; }

/* H.C for a list of rows, by operator algebra (Eq. Haction with the
 * Hamiltonian of Sec. II).  For output row gamma,
 *   (H C)_gamma = sum_beta <gamma|H|beta> C_beta,
 * and each nonzero <gamma|O|beta> is found by applying O^dagger to |gamma>:
 *   O = a+_k a_l                -> O^dagger = a+_l a_k
 *   O = a+_k a+_s a_q a_l       -> O^dagger = a+_l a+_q a_s a_k
 * (operators applied right to left).  All M^2 and M^4 index tuples are
 * visited; tuples whose coefficient is exactly zero are skipped. */
void orc_apply_h_rows(int32_t N, int32_t M, const double *h, const double *g,
                      const double *C, const int64_t *rows, int64_t nrows,
                      double *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < nrows; ++r) {
        int32_t n0[ORC_MAXM], n[ORC_MAXM];
        int64_t gamma = rows[r];
        orc_unhash(N, M, gamma, n0);
        nsum re = {0, 0}, im = {0, 0};
        /* one-body part */
        for (int32_t k = 0; k < M; ++k) {
            for (int32_t l = 0; l < M; ++l) {
                double hr = h[2 * (k * M + l)], hi = h[2 * (k * M + l) + 1];
                if (hr == 0.0 && hi == 0.0) continue;
                memcpy(n, n0, sizeof(int32_t) * M);
                double amp2 = annihilate(n, k);
                if (amp2 == 0.0) continue;
                amp2 *= create(n, l);
                double amp = sqrt(amp2);
                int64_t beta = orc_hash(N, M, n);
                double cr = C[2 * beta], ci = C[2 * beta + 1];
                nadd(&re, amp * (hr * cr - hi * ci));
                nadd(&im, amp * (hr * ci + hi * cr));
            }
        }
        /* two-body part, with the factor 1/2 of the interaction operator */
        for (int32_t k = 0; k < M; ++k)
        for (int32_t s = 0; s < M; ++s)
        for (int32_t q = 0; q < M; ++q)
        for (int32_t l = 0; l < M; ++l) {
            size_t gi = (((size_t)k * M + s) * M + q) * M + l;
            double gr = g[2 * gi], gim = g[2 * gi + 1];
            if (gr == 0.0 && gim == 0.0) continue;
            memcpy(n, n0, sizeof(int32_t) * M);
            double amp2 = annihilate(n, k);
            if (amp2 == 0.0) continue;
            double f = annihilate(n, s);
            if (f == 0.0) continue;
            amp2 *= f;
            amp2 *= create(n, q);
            amp2 *= create(n, l);
            double amp = 0.5 * sqrt(amp2);
            int64_t beta = orc_hash(N, M, n);
            double cr = C[2 * beta], ci = C[2 * beta + 1];
            nadd(&re, amp * (gr * cr - gim * ci));
            nadd(&im, amp * (gr * ci + gim * cr));
        }
        out[2 * r] = nval(&re);
        out[2 * r + 1] = nval(&im);
    }
}

/* Density matrices, Eqs. (rho1) and (rho2):
 *   rho_kl   = sum_gamma conj(C_gamma) <gamma|a+_k a_l|beta> C_beta,
 *   rho_ksql = sum_gamma conj(C_gamma) <gamma|a+_k a+_s a_q a_l|beta> C_beta,
 * with <gamma|O|beta> found, as in H.C, by applying O^dagger to |gamma>.
 * Each configuration gamma is decoded once and visited for every requested
 * element; each thread sums its share of the rows with Neumaier
 * compensation, and the per-thread sums are then added in thread order. */
typedef struct { nsum re, im; } csum;

/* amplitude product of O^dagger applied to n (modified in place), 0 if it
 * annihilates the state; body = 1: a+_l a_k; body = 2: a+_l a+_q a_s a_k */
static double adjoint_string(int32_t *n, int body, int32_t k, int32_t s,
                             int32_t q, int32_t l)
{
    double amp2 = annihilate(n, k);
    if (amp2 == 0.0) return 0.0;
    if (body == 2) {
        double f = annihilate(n, s);
        if (f == 0.0) return 0.0;
        amp2 *= f;
        amp2 *= create(n, q);
    }
    amp2 *= create(n, l);
    return amp2;
}

/* elems[e] = flat element index (k*M + l, or ((k*M + s)*M + q)*M + l) */
static void density_elements(int32_t N, int32_t M, const double *C, int body,
                             const int64_t *elems, int64_t count, double *out)
{
    int64_t D = orc_nc(N, M);
    int nthreads = 1;
#pragma omp parallel
    {
#pragma omp single
        nthreads = omp_get_num_threads();
    }
    csum *part = calloc((size_t)nthreads * (size_t)count, sizeof(csum));
    if (!part) return;
#pragma omp parallel num_threads(nthreads)
    {
        csum *mine = part + (size_t)omp_get_thread_num() * (size_t)count;
        int32_t n0[ORC_MAXM], n[ORC_MAXM];
#pragma omp for schedule(static)
        for (int64_t gamma = 0; gamma < D; ++gamma) {
            orc_unhash(N, M, gamma, n0);
            double ar = C[2 * gamma], ai = -C[2 * gamma + 1];   /* conj(C_gamma) */
            for (int64_t e = 0; e < count; ++e) {
                int64_t t = elems[e];
                int32_t k, s = 0, q = 0, l;
                l = (int32_t)(t % M); t /= M;
                if (body == 2) {
                    q = (int32_t)(t % M); t /= M;
                    s = (int32_t)(t % M); t /= M;
                }
                k = (int32_t)t;
                memcpy(n, n0, sizeof(int32_t) * M);
                double amp2 = adjoint_string(n, body, k, s, q, l);
                if (amp2 == 0.0) continue;
                double amp = sqrt(amp2);
                int64_t beta = orc_hash(N, M, n);
                double br = C[2 * beta], bi = C[2 * beta + 1];
                nadd(&mine[e].re, amp * (ar * br - ai * bi));
                nadd(&mine[e].im, amp * (ar * bi + ai * br));
            }
        }
    }
    for (int64_t e = 0; e < count; ++e) {
        nsum re = {0, 0}, im = {0, 0};
        for (int th = 0; th < nthreads; ++th) {
            nadd(&re, nval(&part[(size_t)th * (size_t)count + (size_t)e].re));
            nadd(&im, nval(&part[(size_t)th * (size_t)count + (size_t)e].im));
        }
        out[2 * e] = nval(&re);
        out[2 * e + 1] = nval(&im);
    }
    free(part);
}

static void density_all(int32_t N, int32_t M, const double *C, int body, double *out)
{
    int64_t count = body == 1 ? (int64_t)M * M : (int64_t)M * M * M * M;
    int64_t *elems = malloc((size_t)count * sizeof(int64_t));
    if (!elems) return;
    for (int64_t e = 0; e < count; ++e) elems[e] = e;
    density_elements(N, M, C, body, elems, count, out);
    free(elems);
}

void orc_rho1(int32_t N, int32_t M, const double *C, double *rho1)
{
    density_all(N, M, C, 1, rho1);
}

/* Selected elements of rho2: idx[e] = ((k*M + s)*M + q)*M + l. */
void orc_rho2_elements(int32_t N, int32_t M, const double *C,
                       const int64_t *idx, int64_t count, double *out)
{
    density_elements(N, M, C, 2, idx, count, out);
}

void orc_rho2(int32_t N, int32_t M, const double *C, double *rho2)
{
    density_all(N, M, C, 2, rho2);
}

/* Occupation vectors of a list of rows (the "hashing table" rows). */
void orc_occ_rows(int32_t N, int32_t M, const int64_t *rows, int64_t nrows,
                  int32_t *occ)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r)
        orc_unhash(N, M, rows[r], occ + r * M);
}

/* Single-jump map (Sec. IV): T1[gamma][k][l] = index of the configuration
 * obtained by moving one particle from orbital k to orbital l, or -1 when
 * orbital k is empty.  For k = l the configuration is unchanged. */
void orc_t1_rows(int32_t N, int32_t M, const int64_t *rows, int64_t nrows,
                 int32_t *t1)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        int32_t n0[ORC_MAXM], n[ORC_MAXM];
        orc_unhash(N, M, rows[r], n0);
        for (int32_t k = 0; k < M; ++k)
            for (int32_t l = 0; l < M; ++l) {
                int32_t *dst = t1 + (r * M + k) * M + l;
                if (n0[k] == 0) { *dst = -1; continue; }
                memcpy(n, n0, sizeof(int32_t) * M);
                n[k] -= 1;
                n[l] += 1;
                *dst = (int32_t)orc_hash(N, M, n);
            }
    }
}

/* Number of valid removal pairs of one configuration (Sec. IV, double-jump
 * map): pairs (k, s) with k <= s, where k = s needs n_k >= 2 and k < s needs
 * n_k >= 1 and n_s >= 1. */
static int64_t removal_pairs(int32_t M, const int32_t *n)
{
    int64_t p = 0;
    for (int32_t k = 0; k < M; ++k)
        for (int32_t s = k; s < M; ++s) {
            if (k == s) { if (n[k] >= 2) ++p; }
            else if (n[k] >= 1 && n[s] >= 1) ++p;
        }
    return p;
}

/* Row lengths of the double-jump map: M^2 entries per valid removal pair. */
void orc_t2_row_lengths(int32_t N, int32_t M, const int64_t *rows,
                        int64_t nrows, int64_t *len)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        int32_t n[ORC_MAXM];
        orc_unhash(N, M, rows[r], n);
        len[r] = removal_pairs(M, n) * (int64_t)M * M;
    }
}

/* Double-jump map rows in the paper's layout (Sec. IV): for each valid
 * removal pair (k, s), k <= s, taken in lexicographic order, a stride of M^2
 * entries; entry q*M + l of the stride is the index of the configuration with
 * one particle removed from k and one from s, then one added to q and one to
 * l.  `offsets[r]` gives where row r starts in `t2` (the caller computes it
 * from orc_t2_row_lengths). */
void orc_t2_rows(int32_t N, int32_t M, const int64_t *rows, int64_t nrows,
                 const int64_t *offsets, int32_t *t2)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        int32_t n0[ORC_MAXM], n[ORC_MAXM];
        orc_unhash(N, M, rows[r], n0);
        int32_t *dst = t2 + offsets[r];
        for (int32_t k = 0; k < M; ++k)
            for (int32_t s = k; s < M; ++s) {
                int valid = (k == s) ? (n0[k] >= 2) : (n0[k] >= 1 && n0[s] >= 1);
                if (!valid) continue;
                for (int32_t q = 0; q < M; ++q)
                    for (int32_t l = 0; l < M; ++l) {
                        memcpy(n, n0, sizeof(int32_t) * M);
                        n[k] -= 1;
                        n[s] -= 1;
                        n[q] += 1;
                        n[l] += 1;
                        *dst++ = (int32_t)orc_hash(N, M, n);
                    }
            }
    }
}

/* Reduced double-jump map: only the true double jumps.  A term
 * a+_q a+_l a_s a_k of the two-body sum whose creation pair {q, l} shares an
 * orbital with the removal pair {k, s} lands on the row itself or on a
 * single jump (the coincident-index cases of the appendix on matrix
 * elements; the footnote on density-matrix cost notes that no index
 * conversion is needed there).  This map keeps the rest: for each valid
 * removal pair (k, s), k <= s, in lexicographic order, the creation pairs
 * (q, l), q <= l, with q and l both outside {k, s}, in lexicographic order;
 * each entry is the index of n - e_k - e_s + e_q + e_l (Eq. TotalCost). */
static int64_t reduced_pair_slots(int32_t M, const int32_t *n)
{
    int64_t c = 0;
    for (int32_t k = 0; k < M; ++k)
        for (int32_t s = k; s < M; ++s) {
            int valid = (k == s) ? (n[k] >= 2) : (n[k] >= 1 && n[s] >= 1);
            if (!valid) continue;
            for (int32_t q = 0; q < M; ++q)
                for (int32_t l = q; l < M; ++l)
                    if (q != k && q != s && l != k && l != s) ++c;
        }
    return c;
}

void orc_t2r_row_lengths(int32_t N, int32_t M, const int64_t *rows,
                         int64_t nrows, int64_t *len)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        int32_t n[ORC_MAXM];
        orc_unhash(N, M, rows[r], n);
        len[r] = reduced_pair_slots(M, n);
    }
}

void orc_t2r_rows(int32_t N, int32_t M, const int64_t *rows, int64_t nrows,
                  const int64_t *offsets, int32_t *t2r)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        int32_t n0[ORC_MAXM], n[ORC_MAXM];
        orc_unhash(N, M, rows[r], n0);
        int32_t *dst = t2r + offsets[r];
        for (int32_t k = 0; k < M; ++k)
            for (int32_t s = k; s < M; ++s) {
                int valid = (k == s) ? (n0[k] >= 2) : (n0[k] >= 1 && n0[s] >= 1);
                if (!valid) continue;
                for (int32_t q = 0; q < M; ++q)
                    for (int32_t l = q; l < M; ++l) {
                        if (q == k || q == s || l == k || l == s) continue;
                        memcpy(n, n0, sizeof(int32_t) * M);
                        n[k] -= 1;
                        n[s] -= 1;
                        n[q] += 1;
                        n[l] += 1;
                        *dst++ = (int32_t)orc_hash(N, M, n);
                    }
            }
    }
}

/* Index of each occupation vector in a list (Eq. TotalCost). */
void orc_hash_rows(int32_t N, int32_t M, const int32_t *occ, int64_t nrows,
                   int64_t *idx)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r)
        idx[r] = orc_hash(N, M, occ + r * M);
}
