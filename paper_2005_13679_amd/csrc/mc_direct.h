// H.C with no table at all: each row's occupations come from its index and
// each jump target from the row's index in closed form.
//
// Summing Eq. (TotalCost) over the particles of each orbital with the
// hockey-stick identity gives the index of an occupation vector n as
//
//   g = D - 1 - sum_{m=0}^{M-2} G_m(S_m),   G_m(S) = C(S + m, m + 1),
//   S_m = n_0 + ... + n_m  (S_{M-1} = N),
//
// a combinatorial number system of degree M-1 in the strictly increasing
// c_m = S_m + m.  So the prefix sums of row g follow greedily from
// J = D - 1 - g (S_m = largest S <= S_{m+1} with G_m(S) <= what is left of J,
// m = M-2 .. 1; G_0(S) = S gives S_0), and a jump changes S_m by
// Delta_m = #{created orbitals <= m} - #{removed orbitals <= m}, a constant
// in {-2..2} for each of the compile-time jumps, so its target is
//
//   t = g + sum_{m: Delta_m != 0} [G_m(S_m) - G_m(S_m + Delta_m)]
//
// with the brackets from a per-row table of (M-1) x 4 integers.  The apply
// reads the staged constants, C (gathers) and nothing else, and writes HC.
// The terms, their constants and their order are those of the case-split
// apply of mc_split.h, so both give the same sums.
//
// Exactness.  D < 2^31 is required.  G_m(x) = P_m(x) / (m+1)! with
// P_m(x) = x (x+1) ... (x+m); for x <= N and m <= M-2, G_m(x) <= D, so
// P_m(x) < 7! 2^31 < 2^44 is exact in double, and the integer G_m(x) is
// recovered exactly by rounding P_m(x) * (1/(m+1)!) (relative error below
// 2^-51 on a value below 2^31).  The greedy step compares P_m(x) with
// J (m+1)! < 2^44, also exact.
#pragma once

#include "mc_split.h"

namespace mc {

__host__ __device__ constexpr double direct_fact(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= (double)i;
    return f;
}

// P_m(x) = x (x+1) ... (x+m), exact for the arguments used here
__device__ __forceinline__ double direct_prod(int m, double x)
{
    double p = x;
#pragma unroll
    for (int i = 1; i < 8; ++i)   // m <= 6 (M <= 8)
        if (i <= m) p *= x + (double)i;
    return p;
}

// G_m(x) = C(x + m, m + 1)
__device__ __forceinline__ double direct_g(int m, double x)
{
    return rint(direct_prod(m, x) * (1.0 / direct_fact(m + 1)));
}

// Prefix sums S_0..S_{M-1} of row `row` (0 <= row < D) of the space of N
// particles: greedily from J = D - 1 - row, S_m = the largest s <= S_{m+1}
// with G_m(s) <= what is left of J, m = M-2 .. 1, then S_0 = the rest.
// `nbits` = bit width of N (a wave-uniform trip count for the search).
template <int MT>
__device__ __forceinline__ void direct_prefix(int64_t row, int64_t D, int N, int nbits,
                                              int (&S)[MT])
{
    S[MT - 1] = N;
    double J = (double)(D - 1 - row);
#pragma unroll
    for (int m = MT - 2; m >= 1; --m) {
        // largest s in [0, S_{m+1}] with P_m(s) <= J (m+1)!  (P_m(0) = 0)
        const double lim = J * direct_fact(m + 1);
        const int hi = S[m + 1];
        int s = 0;
        for (int b = nbits - 1; b >= 0; --b) {
            const int c = s | (1 << b);
            if (c <= hi && direct_prod(m, (double)c) <= lim) s = c;
        }
        S[m] = s;
        J -= direct_g(m, (double)s);
    }
    if constexpr (MT >= 2) S[0] = (int)J;
}

// One row: its index, occupations and the target-index increments.
template <int MT>
struct DirectRow {
    static constexpr int NE = MT > 1 ? MT - 1 : 1;
    uint32_t g;
    int32_t e[NE][4];   // G_m(S_m) - G_m(S_m + d), d = -2, -1, +1, +2 (S_m + d clamped to [0, N])

    // prefix sums of row `row` (0 <= row < D) into S, occupations into n;
    // `nbits` = bit width of N (wave-uniform trip count of the search)
    __device__ __forceinline__ void init(int64_t row, int64_t D, int N, int nbits, int (&n)[MT])
    {
        g = (uint32_t)row;
        int S[MT];
        direct_prefix<MT>(row, D, N, nbits, S);
        n[0] = S[0];
#pragma unroll
        for (int m = 1; m < MT; ++m) n[m] = S[m] - S[m - 1];
#pragma unroll
        for (int m = 0; m + 1 < MT; ++m) {
            const double base = m == 0 ? (double)S[0] : direct_g(m, (double)S[m]);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int d = k < 2 ? k - 2 : k - 1;
                int x = S[m] + d;
                x = x < 0 ? 0 : (x > N ? N : x);
                const double gx = m == 0 ? (double)x : direct_g(m, (double)x);
                e[m][k] = (int32_t)(base - gx);
            }
        }
    }

    template <int M, int D>
    __device__ __forceinline__ uint32_t term() const
    {
        if constexpr (D == 0) return 0u;
        else return (uint32_t)e[M][D < 0 ? D + 2 : D + 1];
    }

    template <int R1, int R2, int A1, int A2, int... Ms>
    __device__ __forceinline__ uint32_t target_fold(std::integer_sequence<int, Ms...>) const
    {
        return (g + ... + term<Ms, prefix_delta(Ms, R1, R2, A1, A2)>());
    }

    // index of the configuration with particles moved from R1, R2 to A1, A2
    template <int R1, int R2, int A1, int A2>
    __device__ __forceinline__ uint32_t target() const
    {
        return target_fold<R1, R2, A1, A2>(std::make_integer_sequence<int, NE>{});
    }
};

// Target of slot U of the case-split stream (the slot order of FlatTile):
// single jump a -> b, or true double jump {K, S} -> {q, l}; -1 where the
// removal is impossible.
template <int MT, int U>
__device__ __forceinline__ int32_t direct_target(const DirectRow<MT> &row, const int (&n)[MT])
{
    constexpr int NSING = FlatTile<MT>::NSING;
    if constexpr (U < NSING) {
        constexpr int a = U / (MT - 1), bb = U % (MT - 1), b = bb + (bb >= a);
        return n[a] >= 1 ? (int32_t)row.template target<a, -1, b, -1>() : -1;
    } else {
        constexpr int e = U - NSING;
        constexpr int P = flat_pair(MT, e), r = flat_slot(MT, e);
        constexpr int K = pair_k(MT, P), S = pair_s(MT, P);
        constexpr int q = reduced_ql(MT, K, S, r, 0), l = reduced_ql(MT, K, S, r, 1);
        const bool valid = K == S ? n[K] >= 2 : (n[K] >= 1 && n[S] >= 1);
        return valid ? (int32_t)row.template target<K, S, q, l>() : -1;
    }
}

// Gathers per basic block (MC_DIRECT_BATCH_WIDE from M = MC_DIRECT_WIDE_FROM
// on, where a tile's 869 windows overrun the caches), and from which M on the
// launch maps blocks to XCD-contiguous ranges of tiles (the L2 of each XCD
// then serves the windows of its own range; measured 6-12 % faster at
// M = 6, 7 and, with the smaller batch, 16 % at M = 8; 1 % slower at M = 5).
#ifndef MC_DIRECT_BATCH
#define MC_DIRECT_BATCH 16
#endif
#ifndef MC_DIRECT_BATCH_WIDE
#define MC_DIRECT_BATCH_WIDE 12
#endif
#ifndef MC_DIRECT_WIDE_FROM
#define MC_DIRECT_WIDE_FROM 8
#endif
#ifndef MC_DIRECT_REMAP_FROM
#define MC_DIRECT_REMAP_FROM 6
#endif

template <int MT>
constexpr bool kDirectRemap = MT >= MC_DIRECT_REMAP_FROM;

template <int MT>
struct DirectStream {
    static constexpr int U = FlatTile<MT>::U;
    static constexpr int B = MT >= MC_DIRECT_WIDE_FROM ? MC_DIRECT_BATCH_WIDE : MC_DIRECT_BATCH;
    static constexpr int SB = U < B ? (U > 0 ? U : 1) : B;
    static constexpr int NB = (U + SB - 1) / SB;
};

template <int MT, bool BIGC, int U0, int... Is>
__device__ __forceinline__ void direct_gathers(std::integer_sequence<int, Is...>,
                                               double2 (&c)[DirectStream<MT>::SB],
                                               const DirectRow<MT> &row, const int (&n)[MT],
                                               const Gather<BIGC> &ldc)
{
    int32_t t[DirectStream<MT>::SB];
    (
        [&] {
            if constexpr (U0 + Is < DirectStream<MT>::U) t[Is] = direct_target<MT, U0 + Is>(row, n);
        }(),
        ...);
    (
        [&] {
            if constexpr (U0 + Is < DirectStream<MT>::U) c[Is] = ldc(t[Is]);
        }(),
        ...);
}

template <int MT, int U0, int... Is>
__device__ __forceinline__ void direct_fmas(std::integer_sequence<int, Is...>,
                                            const double2 (&c)[DirectStream<MT>::SB],
                                            const int (&n)[MT], const RowSq<MT> &R,
                                            const double (&x)[MT], const double2 *__restrict__ HS,
                                            const double2 *__restrict__ GS,
                                            const double2 *__restrict__ GD, double &br,
                                            double &bi, double &ar, double &ai)
{
    (
        [&] {
            if constexpr (U0 + Is < DirectStream<MT>::U)
                flat_fma<MT, U0 + Is>(c[Is], n, R, x, HS, GS, GD, br, bi, ar, ai);
        }(),
        ...);
}

// Batch B of the stream in a basic block of its own (see opaque_true):
// its targets, its gathers, its arithmetic.
template <int MT, bool BIGC, int B>
__device__ __forceinline__ void direct_batches(const DirectRow<MT> &row, const int (&n)[MT],
                                               const RowSq<MT> &R, const double (&x)[MT],
                                               const double2 *__restrict__ HS,
                                               const double2 *__restrict__ GS,
                                               const double2 *__restrict__ GD,
                                               const Gather<BIGC> &ldc, double &br, double &bi,
                                               double &ar, double &ai)
{
    constexpr int SB = DirectStream<MT>::SB, NB = DirectStream<MT>::NB;
    if constexpr (B < NB) {
        if (opaque_true()) {
            double2 c[SB];
            direct_gathers<MT, BIGC, B * SB>(std::make_integer_sequence<int, SB>{}, c, row, n, ldc);
            direct_fmas<MT, B * SB>(std::make_integer_sequence<int, SB>{}, c, n, R, x, HS, GS, GD,
                                    br, bi, ar, ai);
        }
        direct_batches<MT, BIGC, B + 1>(row, n, R, x, HS, GS, GD, ldc, br, bi, ar, ai);
    }
}

// With MC_DIRECT_PIPE: batch B's block first issues batch B+1's gathers
// into the other buffer, then does batch B's arithmetic.
#ifndef MC_DIRECT_PIPE
#define MC_DIRECT_PIPE 0
#endif

template <int MT, bool BIGC, int B>
__device__ __forceinline__ void direct_batches_pipe(double2 (&cur)[DirectStream<MT>::SB],
                                                    double2 (&nxt)[DirectStream<MT>::SB],
                                                    const DirectRow<MT> &row, const int (&n)[MT],
                                                    const RowSq<MT> &R, const double (&x)[MT],
                                                    const double2 *__restrict__ HS,
                                                    const double2 *__restrict__ GS,
                                                    const double2 *__restrict__ GD,
                                                    const Gather<BIGC> &ldc, double &br,
                                                    double &bi, double &ar, double &ai)
{
    constexpr int SB = DirectStream<MT>::SB, NB = DirectStream<MT>::NB;
    if constexpr (B < NB) {
        if (opaque_true()) {
            if constexpr (B + 1 < NB)
                direct_gathers<MT, BIGC, (B + 1) * SB>(std::make_integer_sequence<int, SB>{}, nxt,
                                                       row, n, ldc);
            direct_fmas<MT, B * SB>(std::make_integer_sequence<int, SB>{}, cur, n, R, x, HS, GS,
                                    GD, br, bi, ar, ai);
        }
        direct_batches_pipe<MT, BIGC, B + 1>(nxt, cur, row, n, R, x, HS, GS, GD, ldc, br, bi, ar,
                                             ai);
    }
}

// One 64-row tile of H.C with no table (M <= 8, D < 2^31); `cf` holds the
// constants staged by k_prep_split.
template <int MT, bool BIGC>
__device__ __forceinline__ void apply_tile_direct(int64_t tile, int N, int nbits, int64_t D,
                                                  const double *sq,
                                                  const double2 *__restrict__ cf,
                                                  const double2 *__restrict__ C,
                                                  double2 *__restrict__ HC)
{
    constexpr int M = MT;
    constexpr int P = M * (M + 1) / 2;
    const int lane = threadIdx.x & 63;
    const int64_t g = tile * kTile + lane;
    const bool live = g < D;
    int n[M];
    DirectRow<MT> row;
    row.init(live ? g : D - 1, D, N, nbits, n);
    RowSq<M> R;
    R.init(n, sq);
    double x[M];
#pragma unroll
    for (int m = 0; m < M; ++m) x[m] = (double)n[m];
    const Gather<BIGC> ldc(C, D);
    const double2 *DL = cf + split_dl_offset(M);
    const double2 *GI = cf + split_gi_offset(M);
    const double2 *HS = cf + split_hs_offset(M);
    const double2 *GS = cf + split_gs_offset(M);
    const double2 *GD = cf + split_gd_offset(M);

    // the row's own coefficient (one-body diagonal and coincident pairs)
    const double2 cg = ldc(live ? (int32_t)g : -1);
    double ar, ai;
    {
        double dr = 0.0, di = 0.0;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            dr = fma(DL[k].x, x[k], dr);
            di = fma(DL[k].y, x[k], di);
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const double w = x[pair_k(M, p)] * x[pair_s(M, p)];
            dr = fma(GI[p].x, w, dr);
            di = fma(GI[p].y, w, di);
        }
        ar = dr * cg.x - di * cg.y;
        ai = dr * cg.y + di * cg.x;
    }
    // single jumps, then the true double jumps pair by pair
    double br = 0.0, bi = 0.0;
    if constexpr (MC_DIRECT_PIPE && DirectStream<MT>::NB > 1) {
        double2 ca[DirectStream<MT>::SB], cb[DirectStream<MT>::SB];
        direct_gathers<MT, BIGC, 0>(std::make_integer_sequence<int, DirectStream<MT>::SB>{}, ca,
                                    row, n, ldc);
        direct_batches_pipe<MT, BIGC, 0>(ca, cb, row, n, R, x, HS, GS, GD, ldc, br, bi, ar, ai);
    } else {
        direct_batches<MT, BIGC, 0>(row, n, R, x, HS, GS, GD, ldc, br, bi, ar, ai);
    }
    if (live) HC[g] = make_double2(ar, ai);
}

}  // namespace mc
