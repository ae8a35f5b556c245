// Operators on the coefficient vector through the jump maps:
//   H.C (Eq. Haction with the Hamiltonian of Sec. II), rho1 (Eq. rho1),
//   rho2 (Eq. rho2), and a deterministic complex dot product.
//
// Work decomposition: one wavefront per 64-row tile, lane = row.  For a fixed
// jump slot the 64 lanes read 64 consecutive table entries (one 256-byte
// load) and gather coefficients whose indices are mostly consecutive, since
// the index map is locally affine in the row.  Jump targets of -1 (removal
// from an empty orbital) and padding rows load through a range-checked
// buffer resource and read as zero, so the inner loops have no branches on
// row validity; only the tile-uniform pair mask branches.
#include <utility>

#include "mc_internal.h"

namespace mc {

// Per-call coefficient staging into the workspace:
//   hp[k*M + l]   = h_kl                      (or conj(h_lk) for H^dagger)
//   gp[p*M*M + ql] = G'_{p,ql} = (g_ksql + g_skql)/2 for k < s, g_kkql/2 for
//                    k = s, where p is the index of the removal pair (k, s),
//                    k <= s, in lexicographic order.
// The two ordered removals (k, s) and (s, k) reach the same configuration, so
// their coefficients add; the 1/2 is the interaction prefactor.  For the
// adjoint, g is replaced by g^dagger_ksql = conj(g_lqsk).
__global__ void k_prep(int M, int adjoint, const double2 *__restrict__ g,
                       const double2 *__restrict__ h, double2 *__restrict__ gp,
                       double2 *__restrict__ hp)
{
    const int P = M * (M + 1) / 2;
    const int total = P * M * M;
    auto gat = [&](int k, int s, int q, int l) -> double2 {
        if (!adjoint) return g[((k * M + s) * M + q) * M + l];
        const double2 v = g[((l * M + q) * M + s) * M + k];
        return make_double2(v.x, -v.y);
    };
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total + M * M;
         idx += gridDim.x * blockDim.x) {
        if (idx >= total) {
            const int e = idx - total, k = e / M, l = e % M;
            const double2 v = adjoint ? h[l * M + k] : h[k * M + l];
            hp[e] = make_double2(v.x, adjoint ? -v.y : v.y);
            continue;
        }
        const int p = idx / (M * M), ql = idx % (M * M);
        int k = 0, rem = p;
        while (rem >= M - k) {
            rem -= M - k;
            ++k;
        }
        const int s = k + rem;
        const int q = ql / M, l = ql % M;
        double2 a = gat(k, s, q, l);
        if (k != s) {
            const double2 b = gat(s, k, q, l);
            a.x += b.x;
            a.y += b.y;
        }
        gp[idx] = make_double2(0.5 * a.x, 0.5 * a.y);
    }
}

// Vectors of up to 2^28 entries go through a range-checked buffer resource
// (any t outside [0, D) reads zero); larger ones (BIGC) use 64-bit addresses
// with an explicit range test.
template <bool BIGC>
struct Gather {
    __amdgpu_buffer_rsrc_t r;
    const double2 *__restrict__ p;
    int64_t n;
    __device__ __forceinline__ Gather(const double2 *C, int64_t D)
    {
        p = C;
        n = D;
        if (!BIGC) r = make_rsrc(C, (uint32_t)(D * 16));
    }
    __device__ __forceinline__ double2 operator()(int32_t t) const
    {
        if (!BIGC) return buf_ld_c128(r, (uint32_t)t << 4);
        const bool ok = t >= 0 && t < n;
        const double2 v = p[ok ? t : 0];
        return ok ? v : make_double2(0.0, 0.0);
    }
};

// Per-row square roots of small integers used by the jump amplitudes.
template <int MA>
struct Roots {
    double s0[MA], sm1[MA], sp1[MA], sp2[MA];
};

template <int MT, typename OccT>
__device__ __forceinline__ void load_row(const OccT *__restrict__ occ, int64_t tile, int M,
                                         int lane, int *n, Roots<(MT > 0 ? MT : MC_MAX_M)> &R)
{
    constexpr int MA = MT > 0 ? MT : MC_MAX_M;
#pragma unroll (kUnroll<MT>)
    for (int m = 0; m < MA; ++m) {
        if (MT == 0 && m >= M) break;
        n[m] = (int)occ[(tile * M + m) * kTile + lane];
        const double x = (double)n[m];
        R.s0[m] = sqrt(x);
        R.sm1[m] = sqrt(x > 1.0 ? x - 1.0 : 0.0);
        R.sp1[m] = sqrt(x + 1.0);
        R.sp2[m] = sqrt(x + 2.0);
    }
}

// Removal pair p (lexicographic k <= s) -> (k, s), for compile-time use.
__host__ __device__ constexpr int pair_k(int M, int p)
{
    for (int k = 0; k < M; ++k) {
        if (p < M - k) return k;
        p -= M - k;
    }
    return -1;
}
__host__ __device__ constexpr int pair_s(int M, int p)
{
    for (int k = 0; k < M; ++k) {
        if (p < M - k) return k + p;
        p -= M - k;
    }
    return -1;
}

// Slots of one removal pair handled per batch: a batch issues all its table
// loads, then all its gathers, then the arithmetic.
#ifndef MC_SLOT_BATCH
#define MC_SLOT_BATCH 13
#endif
template <int MT>
constexpr int kSlotBatch = MT * MT < MC_SLOT_BATCH ? MT * MT : MC_SLOT_BATCH;

// Contribution of removal pair P = (K, S), K <= S, to one row:
//   A_KS * sum_{q,l} G'_{P,ql} B_ql(m) C[T2 slot],   m = n - e_K - e_S,
// with `blk` this tile's block of M*M*64 entries for the pair.  Lanes whose
// row cannot lose (K, S) hold -1 entries (gathers read 0) and get A = 0.
template <int MT, bool BIGC, int P>
__device__ __forceinline__ void pair_term(const int32_t *blk, int lane, const int (&n)[MT],
                                          const Roots<MT> &R, const double2 *__restrict__ gp,
                                          const Gather<BIGC> &ldc, double &ar, double &ai)
{
    constexpr int K = pair_k(MT, P), S = pair_s(MT, P);
    constexpr int NS = MT * MT, SB = kSlotBatch<MT>;
    const __amdgpu_buffer_rsrc_t r2 = make_rsrc(blk, (uint32_t)(NS * kTile * 4));
    const bool valid = K == S ? n[K] >= 2 : (n[K] >= 1 && n[S] >= 1);
    const double A = valid ? R.s0[K] * (K == S ? R.sm1[K] : R.s0[S]) : 0.0;
    // creation amplitudes on m: rq = sqrt(m_q + 1), dq = sqrt(m_q + 2)
    double rq[MT], dq[MT];
#pragma unroll
    for (int q = 0; q < MT; ++q) {
        const int d = (q == K) + (q == S);
        rq[q] = d == 0 ? R.sp1[q] : (d == 1 ? R.s0[q] : R.sm1[q]);
        dq[q] = d == 0 ? R.sp2[q] : (d == 1 ? R.sp1[q] : R.s0[q]);
    }
    const double2 *G = gp + P * NS;
    double br = 0.0, bi = 0.0;
#pragma unroll
    for (int j0 = 0; j0 < NS; j0 += SB) {
        int32_t t[SB];
        double2 c[SB];
#pragma unroll
        for (int i = 0; i < SB; ++i)
            if (j0 + i < NS) t[i] = buf_ld_i32(r2, (uint32_t)(((j0 + i) * kTile + lane) * 4), 0);
#pragma unroll
        for (int i = 0; i < SB; ++i)
            if (j0 + i < NS) c[i] = ldc(t[i]);
#pragma unroll
        for (int i = 0; i < SB; ++i) {
            const int j = j0 + i;
            if (j >= NS) break;
            const int q = j / MT, l = j % MT;
            const double B = q == l ? rq[q] * dq[q] : rq[q] * rq[l];
            const double cr = c[i].x * B, ci = c[i].y * B;
            const double2 Gv = G[j];
            br = fma(Gv.x, cr, br);
            br = fma(-Gv.y, ci, br);
            bi = fma(Gv.x, ci, bi);
            bi = fma(Gv.y, cr, bi);
        }
    }
    ar = fma(A, br, ar);
    ai = fma(A, bi, ai);
}

// All removal pairs in order; each present pair is its own basic block
// (uniform branch on the tile's pair mask), which keeps the scheduler from
// hoisting later pairs' loads.
template <int MT, bool BIGC, int... Ps>
__device__ __forceinline__ void all_pairs(std::integer_sequence<int, Ps...>,
                                          const uint64_t *pm, const int32_t *t2, int64_t off0,
                                          int64_t off1, int lane, const int (&n)[MT],
                                          const Roots<MT> &R, const double2 *__restrict__ gp,
                                          const Gather<BIGC> &ldc, double &ar, double &ai)
{
    int64_t pos = off0;
    (
        [&] {
            constexpr int NSB = MT * MT * kTile;
            if (((pm[Ps >> 6] >> (Ps & 63)) & 1) && pos + NSB <= off1) {
                pair_term<MT, BIGC, Ps>(t2 + pos, lane, n, R, gp, ldc, ar, ai);
                pos += NSB;
            }
        }(),
        ...);
}

// H.C for a compile-time orbital count MT (1..8); every orbital, pair and
// slot index is a compile-time constant.
template <int MT, typename OccT, bool BIGC>
__global__ __launch_bounds__(256) void k_apply(int64_t D, int64_t tiles, int64_t nblocks,
                                                int64_t cap, const OccT *__restrict__ occ,
                                                const int32_t *__restrict__ t1,
                                                const uint64_t *__restrict__ pmask,
                                                const int64_t *__restrict__ t2_off,
                                                const int32_t *__restrict__ t2,
                                                const double2 *__restrict__ h,
                                                const double2 *__restrict__ gp,
                                                const double2 *__restrict__ C,
                                                double2 *__restrict__ HC)
{
    constexpr int M = MT;
    constexpr int P = M * (M + 1) / 2;
    constexpr int W = (P + 63) / 64;
    const int lane = threadIdx.x & 63;
    const int64_t tile = xcd_block(blockIdx.x, nblocks) * 4 + wave_in_block();
    if (tile >= tiles) return;
    const int64_t g = tile * kTile + lane;
    const bool live = g < D;

    int n[M];
    Roots<M> R;
    load_row<MT, OccT>(occ, tile, M, lane, n, R);
    const Gather<BIGC> ldc(C, D);

    // diagonal one-body part: sum_k h_kk n_k C_g
    const double2 cg = ldc(live ? (int32_t)g : -1);
    double ar, ai;
    {
        double dr = 0.0, di = 0.0;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const double2 hk = h[k * M + k];
            dr = fma(hk.x, (double)n[k], dr);
            di = fma(hk.y, (double)n[k], di);
        }
        ar = dr * cg.x - di * cg.y;
        ai = dr * cg.y + di * cg.x;
    }

    // single jumps k -> l (k != l): h_kl sqrt(n_k (n_l + 1)) C[T1]
    {
        constexpr int S1 = M * (M - 1);
        const __amdgpu_buffer_rsrc_t r1 =
            make_rsrc(t1 + tile * M * M * kTile, (uint32_t)(M * M * kTile * 4));
        int32_t t[S1 > 0 ? S1 : 1];
        int j = 0;
#pragma unroll
        for (int k = 0; k < M; ++k)
#pragma unroll
            for (int l = 0; l < M; ++l)
                if (l != k) t[j++] = buf_ld_i32(r1, (uint32_t)(((k * M + l) * kTile + lane) * 4), 0);
        double2 c[S1 > 0 ? S1 : 1];
#pragma unroll
        for (int i = 0; i < S1; ++i) c[i] = ldc(t[i]);
        j = 0;
#pragma unroll
        for (int k = 0; k < M; ++k)
#pragma unroll
            for (int l = 0; l < M; ++l) {
                if (l == k) continue;
                const double f = R.s0[k] * R.sp1[l];
                const double2 hv = h[k * M + l];
                const double cr = c[j].x * f, ci = c[j].y * f;
                ++j;
                ar = fma(hv.x, cr, ar);
                ar = fma(-hv.y, ci, ar);
                ai = fma(hv.x, ci, ai);
                ai = fma(hv.y, cr, ai);
            }
    }

    // double jumps: one block of M*M*64 entries per pair present in the tile
    {
        int64_t off0, off1;
        t2_block(t2_off, tile, cap, off0, off1);
        all_pairs<MT, BIGC>(std::make_integer_sequence<int, P>{}, pmask + tile * W, t2, off0, off1,
                            lane, n, R, gp, ldc, ar, ai);
    }
    if (live) HC[g] = make_double2(ar, ai);
}

// ---------------------------------------------------------------------------
// H.C without the double-jump map: a double jump (k, s) -> (q, l) is two
// single jumps, first k -> q from the row, then s -> l from that
// intermediate configuration,
//     T2[g][(k,s)][q*M + l] = T1[T1[g][k][q]][s][l],
// which holds for every valid removal pair (the intermediate still has a
// particle in s).  The tile's single-jump rows stay in registers (they also
// feed the one-body term); the second hop is a gather from rows near g.
// ---------------------------------------------------------------------------
template <int MT, bool BIGC, int P>
__device__ __forceinline__ void pair_term_chained(int64_t D, const int32_t *__restrict__ t1,
                                                  int lane, const int (&n)[MT],
                                                  const Roots<MT> &R,
                                                  const int32_t (&tr)[MT * MT],
                                                  const double2 *__restrict__ gp,
                                                  const Gather<BIGC> &ldc, double &ar,
                                                  double &ai)
{
    constexpr int K = pair_k(MT, P), S = pair_s(MT, P);
    constexpr int NS = MT * MT, SB = kSlotBatch<MT>;
    const bool valid = K == S ? n[K] >= 2 : (n[K] >= 1 && n[S] >= 1);
    if (!__ballot(valid)) return;   // no row of the tile can lose (K, S)
    const double A = valid ? R.s0[K] * (K == S ? R.sm1[K] : R.s0[S]) : 0.0;
    double rq[MT], dq[MT];
#pragma unroll
    for (int q = 0; q < MT; ++q) {
        const int d = (q == K) + (q == S);
        rq[q] = d == 0 ? R.sp1[q] : (d == 1 ? R.s0[q] : R.sm1[q]);
        dq[q] = d == 0 ? R.sp2[q] : (d == 1 ? R.sp1[q] : R.s0[q]);
    }
    const double2 *G = gp + P * NS;
    double br = 0.0, bi = 0.0;
#pragma unroll
    for (int j0 = 0; j0 < NS; j0 += SB) {
        int32_t t[SB];
        double2 c[SB];
#pragma unroll
        for (int i = 0; i < SB; ++i) {
            const int j = j0 + i;
            if (j >= NS) break;
            const int q = j / MT, l = j % MT;
            if (q == K) {
                // first hop k -> k leaves the row unchanged
                t[i] = valid ? tr[S * MT + l] : -1;
            } else {
                const int32_t b = tr[K * MT + q];
                const bool ok = valid && b >= 0 && b < D;
                const int64_t bb = ok ? b : 0;
                const int32_t v = t1[((bb >> 6) * NS + S * MT + l) * kTile + (bb & 63)];
                t[i] = ok ? v : -1;
            }
        }
#pragma unroll
        for (int i = 0; i < SB; ++i)
            if (j0 + i < NS) c[i] = ldc(t[i]);
#pragma unroll
        for (int i = 0; i < SB; ++i) {
            const int j = j0 + i;
            if (j >= NS) break;
            const int q = j / MT, l = j % MT;
            const double B = q == l ? rq[q] * dq[q] : rq[q] * rq[l];
            const double cr = c[i].x * B, ci = c[i].y * B;
            const double2 Gv = G[j];
            br = fma(Gv.x, cr, br);
            br = fma(-Gv.y, ci, br);
            bi = fma(Gv.x, ci, bi);
            bi = fma(Gv.y, cr, bi);
        }
    }
    ar = fma(A, br, ar);
    ai = fma(A, bi, ai);
}

template <int MT, bool BIGC, int... Ps>
__device__ __forceinline__ void all_pairs_chained(std::integer_sequence<int, Ps...>, int64_t D,
                                                  const int32_t *__restrict__ t1, int lane,
                                                  const int (&n)[MT], const Roots<MT> &R,
                                                  const int32_t (&tr)[MT * MT],
                                                  const double2 *__restrict__ gp,
                                                  const Gather<BIGC> &ldc, double &ar,
                                                  double &ai)
{
    (pair_term_chained<MT, BIGC, Ps>(D, t1, lane, n, R, tr, gp, ldc, ar, ai), ...);
}

// One 64-row tile of H.C through single jumps only (see above).
template <int MT, typename OccT, bool BIGC>
__device__ __forceinline__ void apply_tile_chained(int64_t tile, int64_t D,
                                                   const OccT *__restrict__ occ,
                                                   const int32_t *__restrict__ t1,
                                                   const double2 *__restrict__ h,
                                                   const double2 *__restrict__ gp,
                                                   const double2 *__restrict__ C,
                                                   double2 *__restrict__ HC)
{
    constexpr int M = MT;
    constexpr int P = M * (M + 1) / 2;
    const int lane = threadIdx.x & 63;
    const int64_t g = tile * kTile + lane;
    const bool live = g < D;
    int n[M];
    Roots<M> R;
    load_row<MT, OccT>(occ, tile, M, lane, n, R);
    const Gather<BIGC> ldc(C, D);
    int32_t tr[M * M];
    {
        const __amdgpu_buffer_rsrc_t r1 =
            make_rsrc(t1 + tile * M * M * kTile, (uint32_t)(M * M * kTile * 4));
#pragma unroll
        for (int j = 0; j < M * M; ++j) tr[j] = buf_ld_i32(r1, (uint32_t)((j * kTile + lane) * 4), 0);
    }
    const double2 cg = ldc(live ? (int32_t)g : -1);
    double ar, ai;
    {
        double dr = 0.0, di = 0.0;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const double2 hk = h[k * M + k];
            dr = fma(hk.x, (double)n[k], dr);
            di = fma(hk.y, (double)n[k], di);
        }
        ar = dr * cg.x - di * cg.y;
        ai = dr * cg.y + di * cg.x;
    }
    {
        constexpr int S1 = M * (M - 1);
        double2 c[S1 > 0 ? S1 : 1];
        int j = 0;
#pragma unroll
        for (int k = 0; k < M; ++k)
#pragma unroll
            for (int l = 0; l < M; ++l)
                if (l != k) c[j++] = ldc(tr[k * M + l]);
        j = 0;
#pragma unroll
        for (int k = 0; k < M; ++k)
#pragma unroll
            for (int l = 0; l < M; ++l) {
                if (l == k) continue;
                const double f = R.s0[k] * R.sp1[l];
                const double2 hv = h[k * M + l];
                const double cr = c[j].x * f, ci = c[j].y * f;
                ++j;
                ar = fma(hv.x, cr, ar);
                ar = fma(-hv.y, ci, ar);
                ai = fma(hv.x, ci, ai);
                ai = fma(hv.y, cr, ai);
            }
    }
    all_pairs_chained<MT, BIGC>(std::make_integer_sequence<int, P>{}, D, t1, lane, n, R, tr, gp,
                                ldc, ar, ai);
    if (live) HC[g] = make_double2(ar, ai);
}

template <int MT, typename OccT, bool BIGC>
__global__ __launch_bounds__(256) void k_apply_chained(int64_t D, int64_t tiles, int64_t nblocks,
                                                        const OccT *__restrict__ occ,
                                                        const int32_t *__restrict__ t1,
                                                        const double2 *__restrict__ h,
                                                        const double2 *__restrict__ gp,
                                                        const double2 *__restrict__ C,
                                                        double2 *__restrict__ HC)
{
    const int64_t tile = xcd_block(blockIdx.x, nblocks) * 4 + wave_in_block();
    if (tile >= tiles) return;
    apply_tile_chained<MT, OccT, BIGC>(tile, D, occ, t1, h, gp, C, HC);
}

// H.C for any M (run-time orbital loops; the occupations and roots of each
// lane live in LDS so that run-time orbital indices need no register
// indexing).  One wavefront per block; used for M > 8.
template <typename OccT, bool BIGC>
__global__ __launch_bounds__(64) void k_apply_generic(int M, int64_t D, int64_t tiles, int64_t cap,
                                                       const OccT *__restrict__ occ,
                                                       const int32_t *__restrict__ t1,
                                                       const uint64_t *__restrict__ pmask,
                                                       const int64_t *__restrict__ t2_off,
                                                       const int32_t *__restrict__ t2,
                                                       const double2 *__restrict__ h,
                                                       const double2 *__restrict__ gp,
                                                       const double2 *__restrict__ C,
                                                       double2 *__restrict__ HC)
{
    extern __shared__ double sh[];   // [5][M][64]: sqrt(n-1), sqrt(n), sqrt(n+1), sqrt(n+2), n
    const int lane = threadIdx.x;
    const int64_t tile = blockIdx.x;
    if (tile >= tiles) return;
    const int64_t g = tile * kTile + lane;
    const bool live = g < D;
    auto root = [&](int which, int m) -> double { return sh[(which * M + m) * kTile + lane]; };
    for (int m = 0; m < M; ++m) {
        const double x = (double)occ[(tile * M + m) * kTile + lane];
        sh[(0 * M + m) * kTile + lane] = sqrt(x > 1.0 ? x - 1.0 : 0.0);
        sh[(1 * M + m) * kTile + lane] = sqrt(x);
        sh[(2 * M + m) * kTile + lane] = sqrt(x + 1.0);
        sh[(3 * M + m) * kTile + lane] = sqrt(x + 2.0);
        sh[(4 * M + m) * kTile + lane] = x;
    }
    const Gather<BIGC> ldc(C, D);
    const double2 cg = ldc(live ? (int32_t)g : -1);
    double dr = 0.0, di = 0.0;
    for (int k = 0; k < M; ++k) {
        dr += h[k * M + k].x * root(4, k);
        di += h[k * M + k].y * root(4, k);
    }
    double ar = dr * cg.x - di * cg.y, ai = dr * cg.y + di * cg.x;
    const __amdgpu_buffer_rsrc_t r1 =
        make_rsrc(t1 + tile * M * M * kTile, (uint32_t)(M * M * kTile * 4));
    for (int k = 0; k < M; ++k) {
        for (int l = 0; l < M; ++l) {
            if (l == k) continue;
            const int32_t t = buf_ld_i32(r1, lane * 4, (uint32_t)((k * M + l) * kTile * 4));
            const double f = root(1, k) * root(2, l);
            const double2 hv = h[k * M + l];
            const double2 c = ldc(t);
            ar += hv.x * c.x * f - hv.y * c.y * f;
            ai += hv.x * c.y * f + hv.y * c.x * f;
        }
    }
    int64_t off0, off1;
    t2_block(t2_off, tile, cap, off0, off1);
    const __amdgpu_buffer_rsrc_t r2 = make_rsrc(t2 + off0, (uint32_t)((off1 - off0) * 4));
    const int W = (M * (M + 1) / 2 + 63) / 64;
    const uint64_t *pm = pmask + tile * W;
    int rank = 0, p = 0;
    for (int k = 0; k < M; ++k) {
        for (int s = k; s < M; ++s, ++p) {
            if (!((pm[p >> 6] >> (p & 63)) & 1)) continue;
            const double xk = root(4, k), xs = root(4, s);
            const bool valid = k == s ? xk >= 2.0 : (xk >= 1.0 && xs >= 1.0);
            const double A =
                valid ? (k == s ? root(1, k) * root(0, k) : root(1, k) * root(1, s)) : 0.0;
            const double2 *G = gp + p * M * M;
            const uint32_t sbase = (uint32_t)rank * (uint32_t)(M * M * kTile * 4);
            double br = 0.0, bi = 0.0;
            for (int q = 0; q < M; ++q) {
                const int dq_ = (q == k) + (q == s);
                const double rq = root(2 - dq_, q);
                for (int l = 0; l < M; ++l) {
                    const int dl_ = (l == k) + (l == s);
                    const double B = q == l ? rq * root(3 - dq_, q) : rq * root(2 - dl_, l);
                    const int32_t t =
                        buf_ld_i32(r2, lane * 4, sbase + (uint32_t)((q * M + l) * kTile * 4));
                    const double2 c = ldc(t);
                    const double2 Gv = G[q * M + l];
                    br += (Gv.x * c.x - Gv.y * c.y) * B;
                    bi += (Gv.x * c.y + Gv.y * c.x) * B;
                }
            }
            ar += A * br;
            ai += A * bi;
            ++rank;
        }
    }
    if (live) HC[g] = make_double2(ar, ai);
}

// ---------------------------------------------------------------------------
// Density matrices.  Wave w accumulates tiles w, w + nwaves, ... in a fixed
// order; each per-slot value is summed over the 64 rows of the tile with a
// butterfly (all lanes receive the total) and lane (e mod 64) keeps element e.
// Partials per wave go to the workspace and are summed over waves in a fixed
// order by the finalize kernels: results are bitwise reproducible.
// ---------------------------------------------------------------------------
constexpr int kRhoWaves = 4096;

inline int rho_waves(int64_t tiles) { return (int)(tiles < kRhoWaves ? tiles : kRhoWaves); }

template <int MT, typename OccT, bool BIGC>
__global__ __launch_bounds__(256) void k_rho1(int Mrt, int64_t D, int64_t tiles, int nwaves,
                                               const OccT *__restrict__ occ,
                                               const int32_t *__restrict__ t1,
                                               const double2 *__restrict__ C,
                                               double2 *__restrict__ part)
{
    constexpr int MA = MT > 0 ? MT : MC_MAX_M;
    constexpr int NA = (MA * MA + 63) / 64;
    const int M = MT > 0 ? MT : Mrt;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + wave_in_block();
    if (wave >= nwaves) return;
    double accr[NA], acci[NA];
#pragma unroll (kUnroll<MT>)
    for (int j = 0; j < NA; ++j) accr[j] = acci[j] = 0.0;
    const Gather<BIGC> ldc(C, D);
    for (int64_t tile = wave; tile < tiles; tile += nwaves) {
        const int64_t g = tile * kTile + lane;
        int n[MA];
        Roots<MA> R;
        load_row<MT, OccT>(occ, tile, M, lane, n, R);
        const double2 cg = ldc(g < D ? (int32_t)g : -1);
        const __amdgpu_buffer_rsrc_t r1 =
            make_rsrc(t1 + tile * M * M * kTile, (uint32_t)(M * M * kTile * 4));
#pragma unroll (kUnroll<MT>)
        for (int k = 0; k < MA; ++k) {
            if (MT == 0 && k >= M) break;
#pragma unroll (kUnroll<MT>)
            for (int l = 0; l < MA; ++l) {
                if (MT == 0 && l >= M) break;
                double vr, vi;
                if (k == l) {
                    vr = (cg.x * cg.x + cg.y * cg.y) * n[k];
                    vi = 0.0;
                } else {
                    const int32_t t =
                        buf_ld_i32(r1, lane * 4, (uint32_t)((k * M + l) * kTile * 4));
                    const double2 c = ldc(t);
                    const double f = R.s0[k] * R.sp1[l];
                    // conj(C_g) * C_t * f
                    vr = (cg.x * c.x + cg.y * c.y) * f;
                    vi = (cg.x * c.y - cg.y * c.x) * f;
                }
                vr = wave_sum(vr);
                vi = wave_sum(vi);
                const int e = k * M + l;
                if (lane == (e & 63)) {
                    accr[e >> 6] += vr;
                    acci[e >> 6] += vi;
                }
            }
        }
    }
    const int E = M * M;
#pragma unroll (kUnroll<MT>)
    for (int j = 0; j < NA; ++j) {
        const int e = j * 64 + lane;
        if (e < E) part[(int64_t)wave * E + e] = make_double2(accr[j], acci[j]);
    }
}

// One wavefront per block.  Dynamic LDS holds, per lane, the occupations and
// the four root tables of its row ([5][M][64] doubles, private to each lane
// so no barrier is needed) followed by the wave's accumulator of
// E = M(M+1)/2 * M^2 complex elements, updated by lane 0 only.
template <typename OccT, bool BIGC>
__global__ __launch_bounds__(64) void k_rho2(int M, int64_t D, int64_t tiles, int nwaves,
                                              int64_t cap,
                                              const OccT *__restrict__ occ,
                                              const uint64_t *__restrict__ pmask,
                                              const int64_t *__restrict__ t2_off,
                                              const int32_t *__restrict__ t2,
                                              const double2 *__restrict__ C,
                                              double2 *__restrict__ part)
{
    extern __shared__ double sh[];
    const int E = M * (M + 1) / 2 * M * M;
    double *roots = sh;                              // [5][M][64]
    double2 *acc = (double2 *)(sh + 5 * M * kTile);  // [E]
    const int lane = threadIdx.x;
    const int wave = blockIdx.x;
    if (wave >= nwaves) return;
    for (int e = lane; e < E; e += kTile) acc[e] = make_double2(0.0, 0.0);
    __syncthreads();
    const Gather<BIGC> ldc(C, D);
    const int W = (M * (M + 1) / 2 + 63) / 64;
    auto root = [&](int which, int m) -> double { return roots[(which * M + m) * kTile + lane]; };
    for (int64_t tile = wave; tile < tiles; tile += nwaves) {
        const int64_t g = tile * kTile + lane;
        for (int m = 0; m < M; ++m) {
            const double x = (double)occ[(tile * M + m) * kTile + lane];
            roots[(0 * M + m) * kTile + lane] = sqrt(x > 1.0 ? x - 1.0 : 0.0);  // sqrt(n-1)
            roots[(1 * M + m) * kTile + lane] = sqrt(x);                        // sqrt(n)
            roots[(2 * M + m) * kTile + lane] = sqrt(x + 1.0);                  // sqrt(n+1)
            roots[(3 * M + m) * kTile + lane] = sqrt(x + 2.0);                  // sqrt(n+2)
            roots[(4 * M + m) * kTile + lane] = x;                              // n
        }
        const double2 cg = ldc(g < D ? (int32_t)g : -1);
        int64_t off0, off1;
        t2_block(t2_off, tile, cap, off0, off1);
        const __amdgpu_buffer_rsrc_t r2 = make_rsrc(t2 + off0, (uint32_t)((off1 - off0) * 4));
        const uint64_t *pm = pmask + tile * W;
        int rank = 0;
        int p = 0;
        for (int k = 0; k < M; ++k) {
            for (int s = k; s < M; ++s, ++p) {
                const uint64_t word = pm[p >> 6];
                if (!((word >> (p & 63)) & 1)) continue;
                const double xk = root(4, k), xs = root(4, s);
                const bool valid = k == s ? xk >= 2.0 : (xk >= 1.0 && xs >= 1.0);
                const double A =
                    valid ? (k == s ? root(1, k) * root(0, k) : root(1, k) * root(1, s)) : 0.0;
                const uint32_t sbase = (uint32_t)rank * (uint32_t)(M * M * kTile * 4);
                for (int q = 0; q < M; ++q) {
                    // root index of sqrt(m_q + 1) with m = n - e_k - e_s is 2 - d_q
                    const int dq_ = (q == k) + (q == s);
                    const double rq = root(2 - dq_, q);
                    for (int l = 0; l < M; ++l) {
                        const int dl_ = (l == k) + (l == s);
                        const double B = q == l ? rq * root(3 - dq_, q) : rq * root(2 - dl_, l);
                        const int32_t t =
                            buf_ld_i32(r2, lane * 4, sbase + (uint32_t)((q * M + l) * kTile * 4));
                        const double2 c = ldc(t);
                        const double f = A * B;
                        double vr = (cg.x * c.x + cg.y * c.y) * f;
                        double vi = (cg.x * c.y - cg.y * c.x) * f;
                        vr = wave_sum(vr);
                        vi = wave_sum(vi);
                        if (lane == 0) {
                            const int e = p * M * M + q * M + l;
                            acc[e].x += vr;
                            acc[e].y += vi;
                        }
                    }
                }
                ++rank;
            }
        }
    }
    __syncthreads();
    for (int e = lane; e < E; e += kTile) part[(int64_t)wave * E + e] = acc[e];
}

// out[e] = sum over waves of part[w][e], in increasing w.
__global__ void k_rho1_finalize(int E, int nwaves, const double2 *__restrict__ part,
                                double2 *__restrict__ out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double sr = 0.0, si = 0.0;
    for (int w = 0; w < nwaves; ++w) {
        const double2 v = part[(int64_t)w * E + e];
        sr += v.x;
        si += v.y;
    }
    out[e] = make_double2(sr, si);
}

// rho2[k][s][q][l] from the canonical (k <= s) partials.
__global__ void k_rho2_finalize(int M, int nwaves, const double2 *__restrict__ part,
                                double2 *__restrict__ out)
{
    const int total = M * M * M * M;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int l = idx % M, q = (idx / M) % M, s = (idx / (M * M)) % M, k = idx / (M * M * M);
    const int a = k < s ? k : s, b = k < s ? s : k;
    const int p = a * M - a * (a - 1) / 2 + (b - a);
    const int E = M * (M + 1) / 2 * M * M;
    const int e = p * M * M + q * M + l;
    double sr = 0.0, si = 0.0;
    for (int w = 0; w < nwaves; ++w) {
        const double2 v = part[(int64_t)w * E + e];
        sr += v.x;
        si += v.y;
    }
    out[idx] = make_double2(sr, si);
}

// ---------------------------------------------------------------------------
// zdotc: sum_i conj(x_i) y_i with a fixed reduction tree.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_zdotc_partial(int64_t n, const double2 *__restrict__ x,
                                                        const double2 *__restrict__ y,
                                                        double2 *__restrict__ part)
{
    __shared__ double sr[4], si[4];
    double ar = 0.0, ai = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 a = x[i], b = y[i];
        ar += a.x * b.x + a.y * b.y;
        ai += a.x * b.y - a.y * b.x;
    }
    ar = wave_sum(ar);
    ai = wave_sum(ai);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sr[w] = ar;
        si[w] = ai;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        part[blockIdx.x] = make_double2((sr[0] + sr[1]) + (sr[2] + sr[3]),
                                        (si[0] + si[1]) + (si[2] + si[3]));
}

__global__ __launch_bounds__(256) void k_zdotc_final(int nparts, const double2 *__restrict__ part,
                                                      double2 *__restrict__ out)
{
    __shared__ double sr[4], si[4];
    double ar = 0.0, ai = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        ar += part[i].x;
        ai += part[i].y;
    }
    ar = wave_sum(ar);
    ai = wave_sum(ai);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sr[w] = ar;
        si[w] = ai;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        out[0] = make_double2((sr[0] + sr[1]) + (sr[2] + sr[3]), (si[0] + si[1]) + (si[2] + si[3]));
}

// out_i = scale * (op(a) op(x_i) + op(b) op(y_i)); op = conj where flagged;
// a (b) NULL means 1, y NULL drops the second term.
__global__ __launch_bounds__(256) void k_zaxpby(int64_t n, const double2 *__restrict__ a,
                                                 const double2 *__restrict__ x,
                                                 const double2 *__restrict__ b,
                                                 const double2 *__restrict__ y, double scale,
                                                 uint32_t flags, double2 *__restrict__ out)
{
    double2 A = a ? a[0] : make_double2(1.0, 0.0);
    double2 B = b ? b[0] : make_double2(1.0, 0.0);
    if (flags & MC_CONJ_A) A.y = -A.y;
    if (flags & MC_CONJ_B) B.y = -B.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double2 xv = x[i];
        if (flags & MC_CONJ_X) xv.y = -xv.y;
        double rr = A.x * xv.x - A.y * xv.y, ri = A.x * xv.y + A.y * xv.x;
        if (y) {
            double2 yv = y[i];
            if (flags & MC_CONJ_Y) yv.y = -yv.y;
            rr += B.x * yv.x - B.y * yv.y;
            ri += B.x * yv.y + B.y * yv.x;
        }
        out[i] = make_double2(scale * rr, scale * ri);
    }
}

// ---------------------------------------------------------------------------
// Lanczos building blocks with device-resident scalars.
// ---------------------------------------------------------------------------
constexpr int kGemvChunks = 64;

// part[k][b] = sum over chunk b of conj(V_k,i) w_i
__global__ __launch_bounds__(256) void k_zgemv_c_partial(int64_t n, const double2 *__restrict__ V,
                                                          int64_t ldv,
                                                          const double2 *__restrict__ w,
                                                          double2 *__restrict__ part)
{
    __shared__ double sr[4], si[4];
    const int k = blockIdx.y, b = blockIdx.x;
    const int64_t chunk = (n + kGemvChunks - 1) / kGemvChunks;
    const int64_t lo = b * chunk, hi = lo + chunk < n ? lo + chunk : n;
    const double2 *v = V + (int64_t)k * ldv;
    double ar = 0.0, ai = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const double2 a = v[i], c = w[i];
        ar += a.x * c.x + a.y * c.y;
        ai += a.x * c.y - a.y * c.x;
    }
    ar = wave_sum(ar);
    ai = wave_sum(ai);
    if ((threadIdx.x & 63) == 0) {
        sr[threadIdx.x >> 6] = ar;
        si[threadIdx.x >> 6] = ai;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        part[(int64_t)k * kGemvChunks + b] =
            make_double2((sr[0] + sr[1]) + (sr[2] + sr[3]), (si[0] + si[1]) + (si[2] + si[3]));
}

__global__ void k_zgemv_c_final(int K, const double2 *__restrict__ part, double2 *__restrict__ c)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    double sr = 0.0, si = 0.0;
    for (int b = 0; b < kGemvChunks; ++b) {
        sr += part[(int64_t)k * kGemvChunks + b].x;
        si += part[(int64_t)k * kGemvChunks + b].y;
    }
    c[k] = make_double2(sr, si);
}

// w_i -= sum_k V_k,i c_k  (k in increasing order)
__global__ __launch_bounds__(256) void k_zgemv_sub(int K, int64_t n, const double2 *__restrict__ V,
                                                    int64_t ldv, const double2 *__restrict__ c,
                                                    double2 *__restrict__ w)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double sr = 0.0, si = 0.0;
        for (int k = 0; k < K; ++k) {
            const double2 a = V[(int64_t)k * ldv + i], b = c[k];
            sr += a.x * b.x - a.y * b.y;
            si += a.x * b.y + a.y * b.x;
        }
        const double2 x = w[i];
        w[i] = make_double2(x.x - sr, x.y - si);
    }
}

// beta = sqrt(Re <w|w>) from a finished zdotc result; out = w / beta
__global__ __launch_bounds__(256) void k_normalize(int64_t n, const double2 *__restrict__ dot,
                                                   const double2 *__restrict__ w,
                                                   double2 *__restrict__ out,
                                                   double *__restrict__ beta)
{
    const double b = sqrt(dot[0].x);
    if (blockIdx.x == 0 && threadIdx.x == 0 && beta) beta[0] = b;
    const double inv = b > 0.0 ? 1.0 / b : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 x = w[i];
        out[i] = make_double2(x.x * inv, x.y * inv);
    }
}

// w -= Re(alpha) v + beta_prev v_prev (three-term Lanczos recurrence)
__global__ __launch_bounds__(256) void k_lanczos_orth(int64_t n, double2 *__restrict__ w,
                                                       const double2 *__restrict__ v,
                                                       const double2 *__restrict__ vp,
                                                       const double2 *__restrict__ alpha,
                                                       const double *__restrict__ beta_prev)
{
    const double a = alpha[0].x;
    const double b = (vp && beta_prev) ? beta_prev[0] : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double2 x = w[i];
        const double2 y = v[i];
        x.x -= a * y.x;
        x.y -= a * y.y;
        if (b != 0.0) {
            const double2 z = vp[i];
            x.x -= b * z.x;
            x.y -= b * z.y;
        }
        w[i] = x;
    }
}

}  // namespace mc

using namespace mc;

extern "C" {

int mc_lanczos_orth(int64_t n, double *w_d, const double *v_d, const double *vprev_d,
                    const double *alpha_d, const double *beta_prev_d, mc_stream stream)
{
    if (n < 0 || (n > 0 && (!w_d || !v_d || !alpha_d))) return MC_EINVAL;
    if (n == 0) return MC_OK;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_lanczos_orth, dim3(blocks), dim3(256), 0, (hipStream_t)stream, n,
                       (double2 *)w_d, (const double2 *)v_d, (const double2 *)vprev_d,
                       (const double2 *)alpha_d, beta_prev_d);
    return launch_status();
}

int mc_zgemv_c(int32_t K, int64_t n, const double *V_d, int64_t ldv, const double *w_d,
               double *c_d, void *ws_d, size_t ws_bytes, mc_stream stream)
{
    if (K < 0 || n < 0 || ldv < n) return MC_EINVAL;
    if (K == 0) return MC_OK;
    if (!V_d || !w_d || !c_d || !ws_d) return MC_EINVAL;
    if (ws_bytes < (size_t)K * kGemvChunks * 16) return MC_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_zgemv_c_partial, dim3(kGemvChunks, K), dim3(256), 0, s, n,
                       (const double2 *)V_d, ldv, (const double2 *)w_d, (double2 *)ws_d);
    hipLaunchKernelGGL(k_zgemv_c_final, dim3((K + 255) / 256), dim3(256), 0, s, K,
                       (const double2 *)ws_d, (double2 *)c_d);
    return launch_status();
}

int mc_zgemv_sub(int32_t K, int64_t n, const double *V_d, int64_t ldv, const double *c_d,
                 double *w_d, mc_stream stream)
{
    if (K < 0 || n < 0 || ldv < n) return MC_EINVAL;
    if (K == 0 || n == 0) return MC_OK;
    if (!V_d || !w_d || !c_d) return MC_EINVAL;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_zgemv_sub, dim3(blocks), dim3(256), 0, (hipStream_t)stream, K, n,
                       (const double2 *)V_d, ldv, (const double2 *)c_d, (double2 *)w_d);
    return launch_status();
}

int mc_normalize(int64_t n, const double *w_d, double *out_d, double *beta_d, void *ws_d,
                 size_t ws_bytes, mc_stream stream)
{
    if (n < 0 || !w_d || !out_d || !ws_d) return MC_EINVAL;
    if (ws_bytes < (size_t)(MC_DOT_BLOCKS + 2) * 16) return MC_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    double2 *part = (double2 *)ws_d;
    double2 *dot = part + MC_DOT_BLOCKS + 1;
    hipLaunchKernelGGL(k_zdotc_partial, dim3(MC_DOT_BLOCKS), dim3(256), 0, s, n,
                       (const double2 *)w_d, (const double2 *)w_d, part);
    hipLaunchKernelGGL(k_zdotc_final, dim3(1), dim3(256), 0, s, MC_DOT_BLOCKS, part, dot);
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_normalize, dim3(blocks), dim3(256), 0, s, n, dot, (const double2 *)w_d,
                       (double2 *)out_d, beta_d);
    return launch_status();
}

int mc_zaxpby(int64_t n, const double *a_d, const double *x_d, const double *b_d,
              const double *y_d, double scale, uint32_t flags, double *out_d, mc_stream stream)
{
    if (n < 0 || (n > 0 && (!x_d || !out_d))) return MC_EINVAL;
    if (n == 0) return MC_OK;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_zaxpby, dim3(blocks), dim3(256), 0, (hipStream_t)stream, n,
                       (const double2 *)a_d, (const double2 *)x_d, (const double2 *)b_d,
                       (const double2 *)y_d, scale, flags, (double2 *)out_d);
    return launch_status();
}

int mc_workspace_size(int32_t N, int32_t M, int32_t op, size_t *bytes)
{
    if (!bytes) return MC_EINVAL;
    int st = check_nm(N, M);
    if (st) return st;
    const int64_t D = dim_checked(N, M);
    if (D < 0) return MC_ERANGE;
    const int64_t tiles = (D + kTile - 1) / kTile;
    const int64_t P = npairs(M);
    switch (op) {
    case MC_OP_APPLY: *bytes = (size_t)((P * M * M + M * M) * 16); return MC_OK;
    case MC_OP_RHO1: *bytes = (size_t)rho_waves(tiles) * M * M * 16; return MC_OK;
    case MC_OP_RHO2: *bytes = (size_t)rho_waves(tiles) * P * M * M * 16; return MC_OK;
    case MC_OP_DOT: *bytes = (size_t)(MC_DOT_BLOCKS + 1) * 16; return MC_OK;
    default: return MC_EINVAL;
    }
}

static int apply_common(int32_t N, int32_t M, const double *h_d, const double *g_d,
                        const mc_tables *t, const double *C_d, double *HC_d, void *ws_d,
                        size_t ws_bytes, int adjoint, mc_stream stream)
{
    int st = check_nm(N, M);
    if (st) return st;
    const bool chained = t && t->t2_d == nullptr;   // no double-jump map: chain single jumps
    st = check_tables(N, M, t, !chained);
    if (st) return st;
    if (!h_d || !g_d || !C_d || !HC_d || !ws_d) return MC_EINVAL;
    const int64_t D = t->dim;
    if (overlaps(C_d, (size_t)D * 16, HC_d, (size_t)D * 16)) return MC_EINVAL;
    size_t need = 0;
    mc_workspace_size(N, M, MC_OP_APPLY, &need);
    if (ws_bytes < need) return MC_ENOMEM;
    if (M > 8 && (chained || (size_t)5 * M * kTile * 8 > 65536)) return MC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    double2 *gp = (double2 *)ws_d;
    double2 *hp = gp + (size_t)npairs(M) * M * M;
    hipLaunchKernelGGL(k_prep, dim3(4), dim3(256), 0, s, M, adjoint, (const double2 *)g_d,
                       (const double2 *)h_d, gp, hp);
    const int64_t nblocks = (t->tiles + 3) / 4;
    const bool big = D * 16 > (int64_t)0xFFFFFFFFu;
#define MC_APPLY_LAUNCH(OT, BIG)                                                               \
    if (M <= 8) {                                                                              \
        MC_DISPATCH_M(M, if constexpr (MT > 0) hipLaunchKernelGGL(                              \
                             (k_apply<MT, OT, BIG>), dim3(nblocks), dim3(256), 0, s, D,         \
                             t->tiles, nblocks, t->t2_entries, (const OT *)t->occ_d, t->t1_d,   \
                             t->pmask_d, t->t2_off_d, t->t2_d, (const double2 *)hp,             \
                             (const double2 *)gp, (const double2 *)C_d, (double2 *)HC_d));     \
    } else {                                                                                   \
        hipLaunchKernelGGL((k_apply_generic<OT, BIG>), dim3(t->tiles), dim3(64),                \
                           (size_t)5 * M * kTile * 8, s, M, D, t->tiles, t->t2_entries,        \
                           (const OT *)t->occ_d, t->t1_d, t->pmask_d, t->t2_off_d, t->t2_d,    \
                           (const double2 *)hp, (const double2 *)gp, (const double2 *)C_d,     \
                           (double2 *)HC_d);                                                   \
    }
#define MC_CHAINED_LAUNCH(OT, BIG)                                                             \
    MC_DISPATCH_M(M, if constexpr (MT > 0) hipLaunchKernelGGL(                                  \
                         (k_apply_chained<MT, OT, BIG>), dim3(nblocks), dim3(256), 0, s, D,     \
                         t->tiles, nblocks, (const OT *)t->occ_d, t->t1_d, (const double2 *)hp, \
                         (const double2 *)gp, (const double2 *)C_d, (double2 *)HC_d))
    if (chained) {
        if (occ_width(N) == 1) {
            if (big) { MC_CHAINED_LAUNCH(uint8_t, true); } else { MC_CHAINED_LAUNCH(uint8_t, false); }
        } else {
            if (big) { MC_CHAINED_LAUNCH(uint16_t, true); } else { MC_CHAINED_LAUNCH(uint16_t, false); }
        }
    } else if (occ_width(N) == 1) {
        if (big) { MC_APPLY_LAUNCH(uint8_t, true); } else { MC_APPLY_LAUNCH(uint8_t, false); }
    } else {
        if (big) { MC_APPLY_LAUNCH(uint16_t, true); } else { MC_APPLY_LAUNCH(uint16_t, false); }
    }
#undef MC_CHAINED_LAUNCH
#undef MC_APPLY_LAUNCH
    return launch_status();
}

int mc_apply_H(int32_t N, int32_t M, const double *h_d, const double *g_d, const mc_tables *t,
               const double *C_d, double *HC_d, void *ws_d, size_t ws_bytes, mc_stream stream)
{
    return apply_common(N, M, h_d, g_d, t, C_d, HC_d, ws_d, ws_bytes, 0, stream);
}

int mc_apply_H_adjoint(int32_t N, int32_t M, const double *h_d, const double *g_d,
                       const mc_tables *t, const double *C_d, double *HC_d, void *ws_d,
                       size_t ws_bytes, mc_stream stream)
{
    return apply_common(N, M, h_d, g_d, t, C_d, HC_d, ws_d, ws_bytes, 1, stream);
}

int mc_rho1(int32_t N, int32_t M, const mc_tables *t, const double *C_d, double *rho1_d,
            void *ws_d, size_t ws_bytes, mc_stream stream)
{
    int st = check_nm(N, M);
    if (st) return st;
    st = check_tables(N, M, t, false);
    if (st) return st;
    if (!C_d || !rho1_d || !ws_d) return MC_EINVAL;
    size_t need = 0;
    mc_workspace_size(N, M, MC_OP_RHO1, &need);
    if (ws_bytes < need) return MC_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    const int64_t D = t->dim;
    const int nw = rho_waves(t->tiles);
    const bool big = D * 16 > (int64_t)0xFFFFFFFFu;
    double2 *part = (double2 *)ws_d;
#define MC_RHO1_LAUNCH(OT, BIG)                                                               \
    MC_DISPATCH_M(M, hipLaunchKernelGGL((k_rho1<MT, OT, BIG>), dim3((nw + 3) / 4), dim3(256), 0, \
                                        s, M, D, t->tiles, nw, (const OT *)t->occ_d, t->t1_d,  \
                                        (const double2 *)C_d, part))
    if (occ_width(N) == 1) {
        if (big) { MC_RHO1_LAUNCH(uint8_t, true); } else { MC_RHO1_LAUNCH(uint8_t, false); }
    } else {
        if (big) { MC_RHO1_LAUNCH(uint16_t, true); } else { MC_RHO1_LAUNCH(uint16_t, false); }
    }
#undef MC_RHO1_LAUNCH
    const int E = M * M;
    hipLaunchKernelGGL(k_rho1_finalize, dim3((E + 255) / 256), dim3(256), 0, s, E, nw, part,
                       (double2 *)rho1_d);
    return launch_status();
}

int mc_rho2(int32_t N, int32_t M, const mc_tables *t, const double *C_d, double *rho2_d,
            void *ws_d, size_t ws_bytes, mc_stream stream)
{
    int st = check_nm(N, M);
    if (st) return st;
    st = check_tables(N, M, t, true);
    if (st) return st;
    if (!C_d || !rho2_d || !ws_d) return MC_EINVAL;
    size_t need = 0;
    mc_workspace_size(N, M, MC_OP_RHO2, &need);
    if (ws_bytes < need) return MC_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    const int64_t D = t->dim;
    const int nw = rho_waves(t->tiles);
    const bool big = D * 16 > (int64_t)0xFFFFFFFFu;
    double2 *part = (double2 *)ws_d;
#define MC_RHO2_LAUNCH(OT, BIG)                                                          \
    hipLaunchKernelGGL((k_rho2<OT, BIG>), dim3(nw), dim3(64), lds, s, M, D, t->tiles, nw, \
                       t->t2_entries,                                                      \
                       (const OT *)t->occ_d, t->pmask_d, t->t2_off_d, t->t2_d,             \
                       (const double2 *)C_d, part)
    const size_t lds = (size_t)5 * M * kTile * 8 + (size_t)npairs(M) * M * M * 16;
    if (lds > 65536) return MC_EINVAL;   // M <= 8 fits
    if (occ_width(N) == 1) {
        if (big) { MC_RHO2_LAUNCH(uint8_t, true); } else { MC_RHO2_LAUNCH(uint8_t, false); }
    } else {
        if (big) { MC_RHO2_LAUNCH(uint16_t, true); } else { MC_RHO2_LAUNCH(uint16_t, false); }
    }
#undef MC_RHO2_LAUNCH
    const int total = M * M * M * M;
    hipLaunchKernelGGL(k_rho2_finalize, dim3((total + 255) / 256), dim3(256), 0, s, M, nw, part,
                       (double2 *)rho2_d);
    return launch_status();
}

int mc_zdotc(int64_t n, const double *x_d, const double *y_d, double *out_d, void *ws_d,
             size_t ws_bytes, mc_stream stream)
{
    if (n < 0 || !out_d || !ws_d) return MC_EINVAL;
    if (n > 0 && (!x_d || !y_d)) return MC_EINVAL;
    if (ws_bytes < (size_t)(MC_DOT_BLOCKS + 1) * 16) return MC_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    double2 *part = (double2 *)ws_d;
    hipLaunchKernelGGL(k_zdotc_partial, dim3(MC_DOT_BLOCKS), dim3(256), 0, s, n,
                       (const double2 *)x_d, (const double2 *)y_d, part);
    hipLaunchKernelGGL(k_zdotc_final, dim3(1), dim3(256), 0, s, MC_DOT_BLOCKS, part,
                       (double2 *)out_d);
    return launch_status();
}

}  // extern "C"
