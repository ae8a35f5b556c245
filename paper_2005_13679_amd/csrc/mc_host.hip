// Host-side part of the C ABI: status codes, combinatorics, size queries and
// argument validation.  No device work happens here.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "mc_internal.h"

namespace mc {

static thread_local int g_last_hip_error = 0;

int set_hip_error(hipError_t e)
{
    if (e == hipSuccess) return MC_OK;
    g_last_hip_error = (int)e;
    return MC_EHIP;
}

int launch_status() { return set_hip_error(hipGetLastError()); }

int check_nm(int32_t N, int32_t M)
{
    if (M < 1 || M > MC_MAX_M) return MC_EINVAL;
    if (N < 1 || N > MC_MAX_N) return MC_EINVAL;
    return MC_OK;
}

// C(a, b) with 128-bit intermediates; -1 if the result exceeds int64.
static int64_t binom_checked(int64_t a, int64_t b)
{
    if (b < 0 || a < 0 || b > a) return 0;
    if (b > a - b) b = a - b;
    unsigned __int128 r = 1;
    for (int64_t i = 1; i <= b; ++i) {
        r = r * (unsigned __int128)(a - b + i) / (unsigned __int128)i;
        if (r > (unsigned __int128)INT64_MAX) return -1;
    }
    return (int64_t)r;
}

int64_t dim_checked(int32_t N, int32_t M) { return binom_checked((int64_t)N + M - 1, N); }

bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

int check_tables(int32_t N, int32_t M, const mc_tables *t, bool need_t2)
{
    if (!t) return MC_EINVAL;
    if (t->N != N || t->M != M) return MC_EINVAL;
    const int64_t D = dim_checked(N, M);
    if (D <= 0 || t->dim != D) return MC_EINVAL;
    if (t->tiles != (D + kTile - 1) / kTile) return MC_EINVAL;
    if (!t->binom_d || !t->occ_d || !t->t1_d || !t->pmask_d || !t->t2_off_d) return MC_EINVAL;
    if (t->form != MC_FORM_PAPER && t->form != MC_FORM_REDUCED) return MC_EINVAL;
    if (need_t2) {
        if (!t->t2_d || t->t2_required < 0) return MC_EINVAL;
        if (t->t2_entries < t->t2_required) return MC_ENOMEM;
    }
    return MC_OK;
}

}  // namespace mc

using namespace mc;

extern "C" {

const char *mc_strerror(int status)
{
    switch (status) {
    case MC_OK: return "success";
    case MC_EINVAL: return "invalid argument";
    case MC_ERANGE: return "value out of range";
    case MC_ENOMEM: return "buffer or workspace too small";
    case MC_EHIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

int mc_last_hip_error(void) { return g_last_hip_error; }

int64_t mc_dim(int32_t N, int32_t M)
{
    if (N < 0 || M < 1) return MC_EINVAL;
    const int64_t D = dim_checked(N, M);
    return D < 0 ? (int64_t)MC_ERANGE : D;
}

int mc_hash(int32_t N, int32_t M, const int32_t *occ, int64_t *index)
{
    if (!occ || !index || N < 0 || M < 1 || M > MC_MAX_M) return MC_EINVAL;
    int64_t sum = 0;
    for (int m = 0; m < M; ++m) {
        if (occ[m] < 0) return MC_EINVAL;
        sum += occ[m];
    }
    if (sum != N) return MC_EINVAL;
    if (dim_checked(N, M) < 0) return MC_ERANGE;
    int64_t idx = 0;
    int64_t S = occ[0];
    for (int m = 1; m < M; ++m) {
        const int64_t Sp = S;
        S += occ[m];
        idx += binom_checked(S + m, m) - binom_checked(Sp + m, m);
    }
    *index = idx;
    return MC_OK;
}

int mc_unhash(int32_t N, int32_t M, int64_t index, int32_t *occ)
{
    if (!occ || N < 0 || M < 1 || M > MC_MAX_M) return MC_EINVAL;
    const int64_t D = dim_checked(N, M);
    if (D < 0) return MC_ERANGE;
    if (index < 0 || index >= D) return MC_ERANGE;
    int64_t r = index;
    int64_t S = N;
    for (int m = M - 1; m >= 1; --m) {
        const int64_t top = binom_checked(S + m, m);
        const int64_t need = top - r;
        int64_t lo = 0, hi = S;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (binom_checked(mid + m, m) >= need) hi = mid;
            else lo = mid + 1;
        }
        occ[m] = (int32_t)(S - lo);
        r -= top - binom_checked(lo + m, m);
        S = lo;
    }
    occ[0] = (int32_t)S;
    return MC_OK;
}

int mc_tables_size(int32_t N, int32_t M, mc_table_sizes *out)
{
    if (!out) return MC_EINVAL;
    int st = check_nm(N, M);
    if (st) return st;
    const int64_t D = dim_checked(N, M);
    if (D < 0 || D >= ((int64_t)1 << 31)) return MC_ERANGE;
    memset(out, 0, sizeof(*out));
    const int64_t tiles = (D + kTile - 1) / kTile;
    out->dim = D;
    out->tiles = tiles;
    out->occ_bytes = occ_width(N);
    out->pair_words = pair_words(M);
    out->binom_bytes = (int64_t)(N + 3) * (M + 1) * 8;
    out->occ_bytes_total = tiles * M * kTile * out->occ_bytes;
    out->t1_bytes = tiles * M * M * kTile * 4;
    out->pmask_bytes = tiles * out->pair_words * 8;
    out->t2_off_bytes = (tiles + 1) * 8;
    const int64_t pairs_total = N >= 2 ? dim_checked(N - 2, M) : 0;
    out->t2_compact_entries = (int64_t)M * M * npairs(M) * pairs_total;
    out->t2r_compact_entries = reduced_row_entries(M) * pairs_total;
    return MC_OK;
}

// Device bytes of one instance's tables: the sizes above, plus, with the
// double-jump map, its tiled size when every tile holds a block for every
// removal pair (the most it can take: a tile holds a pair's block when any
// of its rows can lose that pair).
int mc_tables_bytes(int32_t N, int32_t M, int32_t form, int32_t with_double_jumps,
                    int64_t *bytes)
{
    if (!bytes) return MC_EINVAL;
    if (form != MC_FORM_PAPER && form != MC_FORM_REDUCED) return MC_EINVAL;
    mc_table_sizes sz;
    const int st = mc_tables_size(N, M, &sz);
    if (st) return st;
    int64_t b = sz.binom_bytes + sz.occ_bytes_total + sz.t1_bytes + sz.pmask_bytes +
                sz.t2_off_bytes;
    if (with_double_jumps) {
        const int64_t per_row = form == MC_FORM_REDUCED ? reduced_row_entries(M)
                                                        : (int64_t)M * M * npairs(M);
        b += 4 * sz.tiles * kTile * per_row;
    }
    *bytes = b;
    return MC_OK;
}

int mc_choose_double_jumps(int32_t count, const int32_t *N, const int32_t *M, int32_t form,
                           double budget_bytes, int32_t *keep)
{
    if (count < 0 || (count > 0 && (!N || !M || !keep))) return MC_EINVAL;
    std::vector<std::pair<int64_t, int32_t>> maps((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        int64_t with = 0, without = 0;
        int st = mc_tables_bytes(N[i], M[i], form, 1, &with);
        if (!st) st = mc_tables_bytes(N[i], M[i], form, 0, &without);
        if (st) return st;
        maps[(size_t)i] = {with - without, i};
        keep[i] = 0;
    }
    std::sort(maps.begin(), maps.end());   // smallest maps first, ties by position
    double left = budget_bytes;
    for (const auto &m : maps) {
        if ((double)m.first > left) break;
        keep[m.second] = 1;
        left -= (double)m.first;
    }
    return MC_OK;
}

// exp(-i T dt) e_0 for the real symmetric tridiagonal T (diagonal alpha[K],
// off-diagonal beta[K-1]): eigen-decomposition T = Q diag(lambda) Q^T by
// cyclic Jacobi rotations (each rotation zeroes one off-diagonal element of
// the symmetric matrix; sweeps repeat until the off-diagonal mass is at
// rounding level), then y = Q exp(-i lambda dt) Q^T e_0.
int mc_tridiag_expv(int32_t K, const double *alpha, const double *beta, double dt, double *y)
{
    if (K < 1 || K > 512 || !alpha || !y || (K > 1 && !beta)) return MC_EINVAL;
    std::vector<double> A((size_t)K * K, 0.0), Q((size_t)K * K, 0.0);
    for (int i = 0; i < K; ++i) {
        A[(size_t)i * K + i] = alpha[i];
        Q[(size_t)i * K + i] = 1.0;
        if (i + 1 < K) A[(size_t)i * K + i + 1] = A[(size_t)(i + 1) * K + i] = beta[i];
    }
    double scale = 0.0;
    for (double v : A) scale += v * v;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < K; ++p)
            for (int q = p + 1; q < K; ++q) off += A[(size_t)p * K + q] * A[(size_t)p * K + q];
        if (off <= 1e-32 * scale) break;
        for (int p = 0; p < K; ++p) {
            for (int q = p + 1; q < K; ++q) {
                const double apq = A[(size_t)p * K + q];
                if (apq == 0.0) continue;
                // rotation (c, s) with tan of the angle t the smaller root of
                // t^2 + 2 theta t - 1 = 0, theta = (a_qq - a_pp) / (2 a_pq)
                const double theta = (A[(size_t)q * K + q] - A[(size_t)p * K + p]) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < K; ++k) {   // A <- A J (columns p, q)
                    const double akp = A[(size_t)k * K + p], akq = A[(size_t)k * K + q];
                    A[(size_t)k * K + p] = c * akp - sn * akq;
                    A[(size_t)k * K + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < K; ++k) {   // A <- J^T A (rows p, q)
                    const double apk = A[(size_t)p * K + k], aqk = A[(size_t)q * K + k];
                    A[(size_t)p * K + k] = c * apk - sn * aqk;
                    A[(size_t)q * K + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < K; ++k) {   // Q <- Q J
                    const double qkp = Q[(size_t)k * K + p], qkq = Q[(size_t)k * K + q];
                    Q[(size_t)k * K + p] = c * qkp - sn * qkq;
                    Q[(size_t)k * K + q] = sn * qkp + c * qkq;
                }
            }
        }
    }
    for (int j = 0; j < K; ++j) {
        double re = 0.0, im = 0.0;
        for (int i = 0; i < K; ++i) {
            const double lam = A[(size_t)i * K + i];
            const double w = Q[(size_t)j * K + i] * Q[i];   // Q[0][i] = Q[i]
            re += w * cos(lam * dt);
            im -= w * sin(lam * dt);
        }
        y[2 * j] = re;
        y[2 * j + 1] = im;
    }
    return MC_OK;
}

// Coefficients of a Short Iterative Lanczos step from its K Lanczos
// coefficients: y = exp(-i T_K dt) e_0, coef = |C| y, and the error
// estimate |C| beta_K |y_{K-1}| (the weight the next Krylov vector would
// get); a vanishing beta_K means an invariant Krylov space and an exact step.
int mc_sil_coefficients(int32_t K, const double *alpha, const double *beta, double beta_next,
                        double norm_c, double dt, double *coef, double *err, int32_t *invariant)
{
    if (!coef || !err || !invariant) return MC_EINVAL;
    const int st = mc_tridiag_expv(K, alpha, beta, dt, coef);
    if (st) return st;
    const double last = hypot(coef[2 * (K - 1)], coef[2 * (K - 1) + 1]);
    *invariant = beta_next < 1e-14 * fmax(1.0, fabs(alpha[K - 1])) ? 1 : 0;
    *err = *invariant ? 0.0 : norm_c * beta_next * last;
    for (int i = 0; i < 2 * K; ++i) coef[i] *= norm_c;
    return MC_OK;
}

// Lowest eigenvalue of the symmetric tridiagonal matrix with diagonal
// alpha[K] and off-diagonal beta[K-1], by bisection on the Sturm count (the
// number of negative pivots of T - x I in its LDL^T factorisation equals the
// number of eigenvalues below x).
int mc_tridiag_lowest(int32_t K, const double *alpha, const double *beta, double *e0)
{
    if (K < 1 || !alpha || !e0 || (K > 1 && !beta)) return MC_EINVAL;
    double lo = alpha[0], hi = alpha[0];
    for (int i = 0; i < K; ++i) {
        const double r = (i > 0 ? fabs(beta[i - 1]) : 0.0) + (i < K - 1 ? fabs(beta[i]) : 0.0);
        lo = fmin(lo, alpha[i] - r);
        hi = fmax(hi, alpha[i] + r);
    }
    const double tiny = 1e-300;
    auto below = [&](double x) {
        int cnt = 0;
        double d = alpha[0] - x;
        if (d < 0) ++cnt;
        for (int i = 1; i < K; ++i) {
            if (fabs(d) < tiny) d = d < 0 ? -tiny : tiny;
            d = alpha[i] - x - beta[i - 1] * beta[i - 1] / d;
            if (d < 0) ++cnt;
        }
        return cnt;
    };
    for (int it = 0; it < 200 && hi - lo > 0; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (below(mid) >= 1) hi = mid;
        else lo = mid;
    }
    *e0 = 0.5 * (lo + hi);
    return MC_OK;
}

}  // extern "C"
