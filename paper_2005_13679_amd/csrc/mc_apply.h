// Device-side building blocks of H.C (Eq. Haction) shared by the plain and
// batched kernels: one 64-row tile per wavefront, lane = row, through either
// the double-jump map or two chained single jumps.
#pragma once

#include <utility>

#include "mc_internal.h"

#ifndef MC_SLOT_BATCH
#define MC_SLOT_BATCH 13
#endif
// Occupancy the apply kernels are compiled for (wavefronts per SIMD); the
// register allocator caps VGPRs accordingly (512 / waves).
#ifndef MC_APPLY_WAVES
#define MC_APPLY_WAVES 2
#endif
// Double-jump index loads: 0 = each batch loads its indices, then gathers;
// 1 = the next batch's indices are loaded while the current batch's gathers
// are in flight (within a pair); 2 = also the first batch of the next block
// (across pairs, and the first block during the one-body part).
#ifndef MC_T2_PIPELINE
#define MC_T2_PIPELINE 0
#endif

namespace mc {

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

// Per-row square roots of small integers used by the jump amplitudes:
// root<d>(m) = sqrt(n_m + d) for d in {-1, 0, 1, 2} (0 where n_m + d < 0).
// Either the four tables live in registers (8M VGPRs), or only the
// occupations do and the roots come from an LDS table of sqrt(i),
// i = 0 .. N+2, filled once per block: from M = 5 on, where the registers
// are worth more as waves in flight.
#ifndef MC_LDS_ROOTS_FROM
#define MC_LDS_ROOTS_FROM 5
#endif
template <int MT>
constexpr bool kLdsRoots = MT >= MC_LDS_ROOTS_FROM;
// The chained paper-form body keeps its roots in registers up to M = 5
// (measured: the LDS table slowed it by a fifth at M = 5, while it sped the
// map and case-split bodies up by 2-6 %, their registers going to waves).
template <int MT>
constexpr bool kLdsRootsChained = MT >= 6;

template <int MT, bool LDS = kLdsRoots<MT>>
struct RowSq;

template <int MT>
struct RowSq<MT, false> {
    double sm1[MT], s0[MT], sp1[MT], sp2[MT];
    __device__ __forceinline__ void init(const int (&n)[MT], const double *)
    {
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const double x = (double)n[m];
            s0[m] = sqrt(x);
            sm1[m] = sqrt(x > 1.0 ? x - 1.0 : 0.0);
            sp1[m] = sqrt(x + 1.0);
            sp2[m] = sqrt(x + 2.0);
        }
    }
    template <int d>
    __device__ __forceinline__ double root(int m) const
    {
        static_assert(d >= -1 && d <= 2, "root offset");
        return d == -1 ? sm1[m] : (d == 0 ? s0[m] : (d == 1 ? sp1[m] : sp2[m]));
    }
};

template <int MT>
struct RowSq<MT, true> {
    int nn[MT];
    const double *sq;
    __device__ __forceinline__ void init(const int (&n)[MT], const double *tab)
    {
#pragma unroll
        for (int m = 0; m < MT; ++m) nn[m] = n[m];
        sq = tab;
    }
    template <int d>
    __device__ __forceinline__ double root(int m) const
    {
        const int i = nn[m] + d;
        return sq[i > 0 ? i : 0];
    }
};

// sqrt(i) for i = 0 .. n-1 into LDS (block-wide; every thread must call it)
__device__ __forceinline__ void fill_sqrt_table(double *tab, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) tab[i] = sqrt((double)i);
    __syncthreads();
}

template <int MT, typename OccT, bool LDS>
__device__ __forceinline__ void load_row(const OccT *__restrict__ occ, int64_t tile, int lane,
                                         int (&n)[MT], RowSq<MT, LDS> &R, const double *sq)
{
#pragma unroll
    for (int m = 0; m < MT; ++m) n[m] = (int)occ[(tile * MT + m) * kTile + lane];
    R.init(n, sq);
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
template <int MT>
constexpr int kSlotBatch = MT * MT < MC_SLOT_BATCH ? MT * MT : MC_SLOT_BATCH;
// Double-jump blocks of the paper form: a whole M*M block per batch up to
// M * M = MC_T2_WHOLE_BLOCK (larger M would spill).
#ifndef MC_T2_WHOLE_BLOCK
#define MC_T2_WHOLE_BLOCK 25
#endif
template <int MT>
constexpr int kT2Batch = MT * MT <= MC_T2_WHOLE_BLOCK ? MT * MT : kSlotBatch<MT>;

// The paper's double-jump block holds one column per ordered creation pair
// (q, l); (q, l) and (l, q) reach one configuration, so the per-pair walk
// reads the columns with q <= l only and weights them by G'_{P,ql} +
// G'_{P,lq}.  Slot j of the walk is column t2_col(j) of the block.
#ifndef MC_PAPER_TRIANGLE
#define MC_PAPER_TRIANGLE 1
#endif
template <int MT>
constexpr int kT2Slots = MC_PAPER_TRIANGLE ? MT * (MT + 1) / 2 : MT * MT;

template <int MT>
__host__ __device__ constexpr int t2_col(int j)
{
    if (!MC_PAPER_TRIANGLE) return j;
    for (int q = 0; q < MT; ++q) {
        if (j < MT - q) return q * MT + q + j;
        j -= MT - q;
    }
    return 0;
}

// Indices of walk slots [J0, J0 + SB) of a double-jump block (one per lane).
template <int MT, int SB, int J0>
__device__ __forceinline__ void load_t2_batch(int32_t (&t)[SB], __amdgpu_buffer_rsrc_t r, int lane)
{
#pragma unroll
    for (int i = 0; i < SB; ++i)
        if (J0 + i < kT2Slots<MT>)
            t[i] = buf_ld_i32(r, (uint32_t)((t2_col<MT>(J0 + i) * kTile + lane) * 4), 0);
}

// Resource over the double-jump block starting at `pos`, clipped to the
// tile's [., off1) range (a zero-length resource makes loads return 0).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t t2_block_rsrc(const int32_t *t2, int64_t pos,
                                                                int64_t off1, int ns)
{
    int64_t n = off1 - pos;
    n = n < 0 ? 0 : (n > (int64_t)ns * kTile ? (int64_t)ns * kTile : n);
    return make_rsrc(t2 + (pos < off1 ? pos : off1), (uint32_t)(n * 4));
}

// Contribution of removal pair P = (K, S), K <= S, to one row:
//   A_KS * sum_{q,l} G'_{P,ql} B_ql(m) C[T2 slot],   m = n - e_K - e_S,
// for the pair's block at `pos` (M*M*64 entries).  Lanes whose row cannot
// lose (K, S) hold -1 entries (gathers read 0) and get A = 0.
// Software pipeline: `tf` holds the first index batch of this block on entry
// (loaded earlier); batch b's gathers are issued, then the next batch's
// indices are loaded (after the last batch: the first batch of the next
// block, which is simply the next M*M*64 entries since the blocks of the
// present pairs are contiguous), then batch b's arithmetic waits for its
// gathers.
template <int MT, bool BIGC, int B, int NB>
__device__ __forceinline__ void pair_batches(const int32_t *t2, int64_t pos, int64_t off1, int lane,
                                             __amdgpu_buffer_rsrc_t r2,
                                             int32_t (&tf)[kT2Batch<MT>],
                                             int32_t (&tn)[kT2Batch<MT>], const double (&rq)[MT],
                                             const double (&dq)[MT], const double2 *__restrict__ G,
                                             const Gather<BIGC> &ldc, double &br, double &bi)
{
    if constexpr (B < NB) {
        constexpr int NS = kT2Slots<MT>, SB = kT2Batch<MT>, J0 = B * SB;
        double2 c[SB];
        if constexpr (MC_T2_PIPELINE == 0) {
            // indices of this batch, then its gathers
            load_t2_batch<MT, SB, J0>(tn, r2, lane);
#pragma unroll
            for (int i = 0; i < SB; ++i)
                if (J0 + i < NS) c[i] = ldc(tn[i]);
        } else {
            if constexpr (MC_T2_PIPELINE == 1 && B == 0) load_t2_batch<MT, SB, 0>(tf, r2, lane);
#pragma unroll
            for (int i = 0; i < SB; ++i)
                if (J0 + i < NS) c[i] = ldc(B == 0 ? tf[i] : tn[i]);
            if constexpr (B + 1 < NB) {
                load_t2_batch<MT, SB, J0 + SB>(tn, r2, lane);
            } else if constexpr (MC_T2_PIPELINE == 2) {
                const __amdgpu_buffer_rsrc_t rn =
                    t2_block_rsrc(t2, pos + MT * MT * kTile, off1, MT * MT);
                load_t2_batch<MT, SB, 0>(tf, rn, lane);
            }
        }
#pragma unroll
        for (int i = 0; i < SB; ++i) {
            const int j = J0 + i;
            if (j >= NS) break;
            const int col = t2_col<MT>(j), q = col / MT, l = col % MT;
            const double Bf = q == l ? rq[q] * dq[q] : rq[q] * rq[l];
            const double cr = c[i].x * Bf, ci = c[i].y * Bf;
            double2 Gv = G[col];
            if (MC_PAPER_TRIANGLE && q != l) {
                Gv.x += G[l * MT + q].x;
                Gv.y += G[l * MT + q].y;
            }
            br = fma(Gv.x, cr, br);
            br = fma(-Gv.y, ci, br);
            bi = fma(Gv.x, ci, bi);
            bi = fma(Gv.y, cr, bi);
        }
        pair_batches<MT, BIGC, B + 1, NB>(t2, pos, off1, lane, r2, tf, tn, rq, dq, G, ldc, br, bi);
    }
}

template <int MT, bool BIGC, int P>
__device__ __forceinline__ void pair_term(const int32_t *t2, int64_t pos, int64_t off1, int lane,
                                          const int (&n)[MT], const RowSq<MT> &R,
                                          const double2 *__restrict__ gp, const Gather<BIGC> &ldc,
                                          int32_t (&tf)[kT2Batch<MT>], double &ar, double &ai)
{
    constexpr int K = pair_k(MT, P), S = pair_s(MT, P);
    constexpr int NS = MT * MT, SB = kT2Batch<MT>;
    constexpr int NB = (kT2Slots<MT> + SB - 1) / SB;
    const __amdgpu_buffer_rsrc_t r2 = make_rsrc(t2 + pos, (uint32_t)(NS * kTile * 4));
    const bool valid = K == S ? n[K] >= 2 : (n[K] >= 1 && n[S] >= 1);
    const double A =
        valid ? R.template root<0>(K) * (K == S ? R.template root<-1>(K) : R.template root<0>(S))
              : 0.0;
    // creation amplitudes on m: rq = sqrt(m_q + 1), dq = sqrt(m_q + 2)
    double rq[MT], dq[MT];
#pragma unroll
    for (int q = 0; q < MT; ++q) {
        const int d = (q == K) + (q == S);
        rq[q] = d == 0 ? R.template root<1>(q) : (d == 1 ? R.template root<0>(q) : R.template root<-1>(q));
        dq[q] = d == 0 ? R.template root<2>(q) : (d == 1 ? R.template root<1>(q) : R.template root<0>(q));
    }
    int32_t tn[SB];
    double br = 0.0, bi = 0.0;
    pair_batches<MT, BIGC, 0, NB>(t2, pos, off1, lane, r2, tf, tn, rq, dq, gp + P * NS, ldc, br, bi);
    ar = fma(A, br, ar);
    ai = fma(A, bi, ai);
}

// All removal pairs in order; each present pair is its own basic block
// (uniform branch on the tile's pair mask), which keeps the scheduler from
// hoisting later pairs' loads.  `tf` carries the prefetched first index
// batch of the next block from pair to pair.
template <int MT, bool BIGC, int... Ps>
__device__ __forceinline__ void all_pairs(std::integer_sequence<int, Ps...>,
                                          const uint64_t *pm, const int32_t *t2, int64_t off0,
                                          int64_t off1, int lane, const int (&n)[MT],
                                          const RowSq<MT> &R, const double2 *__restrict__ gp,
                                          const Gather<BIGC> &ldc, int32_t (&tf)[kT2Batch<MT>],
                                          double &ar, double &ai)
{
    int64_t pos = off0;
    (
        [&] {
            constexpr int NSB = MT * MT * kTile;
            if (((pm[Ps >> 6] >> (Ps & 63)) & 1) && pos + NSB <= off1) {
                pair_term<MT, BIGC, Ps>(t2, pos, off1, lane, n, R, gp, ldc, tf, ar, ai);
                pos += NSB;
            }
        }(),
        ...);
}

// One 64-row tile of H.C for a compile-time orbital count MT (1..8) through
// the single- and double-jump maps; every orbital, pair and slot index is a
// compile-time constant.  Called by one whole wavefront.
template <int MT, typename OccT, bool BIGC>
__device__ __forceinline__ void apply_tile_t2(int64_t tile, int64_t D, int64_t cap, const double *sq,
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
    constexpr int M = MT;
    constexpr int P = M * (M + 1) / 2;
    constexpr int W = (P + 63) / 64;
    const int lane = threadIdx.x & 63;
    const int64_t g = tile * kTile + lane;
    const bool live = g < D;

    // first index batch of the tile's first double-jump block, in flight
    // during the one-body part
    int64_t off0, off1;
    t2_block(t2_off, tile, cap, off0, off1);
    int32_t tf[kT2Batch<MT>];
    if constexpr (MC_T2_PIPELINE == 2)
        load_t2_batch<MT, kT2Batch<MT>, 0>(tf, t2_block_rsrc(t2, off0, off1, M * M), lane);

    int n[M];
    RowSq<M> R;
    load_row<MT, OccT>(occ, tile, lane, n, R, sq);
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

    // single jumps k -> l (k != l): h_kl sqrt(n_k (n_l + 1)) C[T1], in
    // batches of kSlotBatch slots (table loads, then gathers, then FMAs)
    {
        constexpr int NS = M * M, SB = kSlotBatch<MT>;
        const __amdgpu_buffer_rsrc_t r1 =
            make_rsrc(t1 + tile * NS * kTile, (uint32_t)(NS * kTile * 4));
#pragma unroll
        for (int j0 = 0; j0 < NS; j0 += SB) {
            int32_t t[SB];
            double2 c[SB];
#pragma unroll
            for (int i = 0; i < SB; ++i) {
                const int j = j0 + i;
                if (j < NS && j / M != j % M)
                    t[i] = buf_ld_i32(r1, (uint32_t)((j * kTile + lane) * 4), 0);
            }
#pragma unroll
            for (int i = 0; i < SB; ++i) {
                const int j = j0 + i;
                if (j < NS && j / M != j % M) c[i] = ldc(t[i]);
            }
#pragma unroll
            for (int i = 0; i < SB; ++i) {
                const int j = j0 + i;
                if (j >= NS) break;
                const int k = j / M, l = j % M;
                if (k == l) continue;
                const double f = R.template root<0>(k) * R.template root<1>(l);
                const double2 hv = h[j];
                const double cr = c[i].x * f, ci = c[i].y * f;
                ar = fma(hv.x, cr, ar);
                ar = fma(-hv.y, ci, ar);
                ai = fma(hv.x, ci, ai);
                ai = fma(hv.y, cr, ai);
            }
        }
    }

    // double jumps: one block of M*M*64 entries per pair present in the tile
    all_pairs<MT, BIGC>(std::make_integer_sequence<int, P>{}, pmask + tile * W, t2, off0, off1,
                        lane, n, R, gp, ldc, tf, ar, ai);
    if (live) HC[g] = make_double2(ar, ai);
}


// ---------------------------------------------------------------------------
// H.C without the double-jump map: a double jump (k, s) -> (q, l) is two
// single jumps, first k -> q from the row, then s -> l from that
// intermediate configuration,
//     T2[g][(k,s)][q*M + l] = T1[T1[g][k][q]][s][l],
// which holds for every valid removal pair (the intermediate still has a
// particle in s).  For q = k the first hop leaves the row unchanged and the
// target is the single jump T1[g][s][l].  First hops and q = k targets come
// from the tile's own single-jump block (coalesced, cache-resident); the
// second hop is a gather from rows near g.
// ---------------------------------------------------------------------------
template <int MT, bool BIGC, int P>
__device__ __forceinline__ void pair_term_chained(int64_t D, const int32_t *__restrict__ t1,
                                                  __amdgpu_buffer_rsrc_t r1, int lane,
                                                  const int (&n)[MT], const RowSq<MT, kLdsRootsChained<MT>> &R,
                                                  const double2 *__restrict__ gp,
                                                  const Gather<BIGC> &ldc, double &ar, double &ai)
{
    constexpr int K = pair_k(MT, P), S = pair_s(MT, P);
    constexpr int NS = MT * MT, SB = kSlotBatch<MT>;
    const bool valid = K == S ? n[K] >= 2 : (n[K] >= 1 && n[S] >= 1);
    if (!__ballot(valid)) return;   // no row of the tile can lose (K, S)
    const double A =
        valid ? R.template root<0>(K) * (K == S ? R.template root<-1>(K) : R.template root<0>(S))
              : 0.0;
    double rq[MT], dq[MT];
#pragma unroll
    for (int q = 0; q < MT; ++q) {
        const int d = (q == K) + (q == S);
        rq[q] = d == 0 ? R.template root<1>(q) : (d == 1 ? R.template root<0>(q) : R.template root<-1>(q));
        dq[q] = d == 0 ? R.template root<2>(q) : (d == 1 ? R.template root<1>(q) : R.template root<0>(q));
    }
    // first hops K -> q of this row
    int32_t fh[MT];
#pragma unroll
    for (int q = 0; q < MT; ++q)
        fh[q] = q == K ? 0 : buf_ld_i32(r1, (uint32_t)(((K * MT + q) * kTile + lane) * 4), 0);
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
                const int32_t v = buf_ld_i32(r1, (uint32_t)(((S * MT + l) * kTile + lane) * 4), 0);
                t[i] = valid ? v : -1;
            } else {
                const int32_t b = fh[q];
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

// The same double jumps for M >= 6 with the removal pairs as a loop: the
// compile-time fold over M(M+1)/2 pairs of M^2 slots each keeps too many
// values live at once there.  K and S are wave-uniform loop counters; q and
// l stay compile-time, so the per-row occupations are picked with selects and
// the roots come from the block's sqrt table.
template <int MT, bool BIGC>
__device__ __forceinline__ void pairs_chained_loop(int64_t D, int64_t g,
                                                   const int32_t *__restrict__ t1,
                                                   __amdgpu_buffer_rsrc_t r1, int lane,
                                                   const int (&n)[MT], const double *sq,
                                                   const double2 *__restrict__ gp,
                                                   const Gather<BIGC> &ldc, double &ar, double &ai)
{
    constexpr int NS = MT * MT, SB = kSlotBatch<MT>;
    int P = 0;
#pragma unroll 1
    for (int K = 0; K < MT; ++K) {
#pragma unroll 1
        for (int S = K; S < MT; ++S, ++P) {
            int nK = 0, nS = 0;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                nK = m == K ? n[m] : nK;
                nS = m == S ? n[m] : nS;
            }
            const bool valid = K == S ? nK >= 2 : (nK >= 1 && nS >= 1);
            if (!__ballot(valid)) continue;
            const double A = valid ? sq[nK] * (K == S ? sq[nK > 0 ? nK - 1 : 0] : sq[nS]) : 0.0;
            // first hops K -> q (q = K: the row itself)
            int32_t b[MT];
#pragma unroll
            for (int q = 0; q < MT; ++q) {
                const int32_t f = buf_ld_i32(r1, (uint32_t)(((K * MT + q) * kTile + lane) * 4), 0);
                b[q] = q == K ? (int32_t)g : f;
            }
            double rq[MT];
#pragma unroll
            for (int q = 0; q < MT; ++q) {
                const int i = n[q] + 1 - (q == K) - (q == S);
                rq[q] = sq[i > 0 ? i : 0];
            }
            const double2 *G = gp + (int64_t)P * NS;
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
                    const int32_t bq = b[q];
                    const bool ok = valid && bq >= 0 && bq < D;
                    const int64_t bb = ok ? bq : 0;
                    const int32_t v = t1[((bb >> 6) * NS + S * MT + l) * kTile + (bb & 63)];
                    t[i] = ok ? v : -1;
                }
#pragma unroll
                for (int i = 0; i < SB; ++i)
                    if (j0 + i < NS) c[i] = ldc(t[i]);
#pragma unroll
                for (int i = 0; i < SB; ++i) {
                    const int j = j0 + i;
                    if (j >= NS) break;
                    const int q = j / MT, l = j % MT;
                    double Bv;
                    if (q == l) {
                        const int i2 = n[q] + 2 - (q == K) - (q == S);
                        Bv = rq[q] * sq[i2 > 0 ? i2 : 0];
                    } else {
                        Bv = rq[q] * rq[l];
                    }
                    const double cr = c[i].x * Bv, ci = c[i].y * Bv;
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
    }
}

template <int MT, bool BIGC, int... Ps>
__device__ __forceinline__ void all_pairs_chained(std::integer_sequence<int, Ps...>, int64_t D,
                                                  const int32_t *__restrict__ t1,
                                                  __amdgpu_buffer_rsrc_t r1, int lane,
                                                  const int (&n)[MT], const RowSq<MT, kLdsRootsChained<MT>> &R,
                                                  const double2 *__restrict__ gp,
                                                  const Gather<BIGC> &ldc, double &ar, double &ai)
{
    (pair_term_chained<MT, BIGC, Ps>(D, t1, r1, lane, n, R, gp, ldc, ar, ai), ...);
}

// One 64-row tile of H.C through single jumps only (see above).
template <int MT, typename OccT, bool BIGC>
__device__ __forceinline__ void apply_tile_chained(int64_t tile, int64_t D, const double *sq,
                                                   const OccT *__restrict__ occ,
                                                   const int32_t *__restrict__ t1,
                                                   const double2 *__restrict__ h,
                                                   const double2 *__restrict__ gp,
                                                   const double2 *__restrict__ C,
                                                   double2 *__restrict__ HC)
{
    constexpr int M = MT;
    constexpr int P = M * (M + 1) / 2;
    constexpr int NS = M * M, SB = kSlotBatch<MT>;
    const int lane = threadIdx.x & 63;
    const int64_t g = tile * kTile + lane;
    const bool live = g < D;
    int n[M];
    RowSq<M, kLdsRootsChained<MT>> R;
    load_row<MT, OccT>(occ, tile, lane, n, R, sq);
    const Gather<BIGC> ldc(C, D);
    const __amdgpu_buffer_rsrc_t r1 =
        make_rsrc(t1 + tile * NS * kTile, (uint32_t)(NS * kTile * 4));
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
    // single jumps k -> l (k != l), in batches
#pragma unroll
    for (int j0 = 0; j0 < NS; j0 += SB) {
        int32_t t[SB];
        double2 c[SB];
#pragma unroll
        for (int i = 0; i < SB; ++i) {
            const int j = j0 + i;
            if (j < NS && j / M != j % M) t[i] = buf_ld_i32(r1, (uint32_t)((j * kTile + lane) * 4), 0);
        }
#pragma unroll
        for (int i = 0; i < SB; ++i) {
            const int j = j0 + i;
            if (j < NS && j / M != j % M) c[i] = ldc(t[i]);
        }
#pragma unroll
        for (int i = 0; i < SB; ++i) {
            const int j = j0 + i;
            if (j >= NS) break;
            const int k = j / M, l = j % M;
            if (k == l) continue;
            const double f = R.template root<0>(k) * R.template root<1>(l);
            const double2 hv = h[j];
            const double cr = c[i].x * f, ci = c[i].y * f;
            ar = fma(hv.x, cr, ar);
            ar = fma(-hv.y, ci, ar);
            ai = fma(hv.x, ci, ai);
            ai = fma(hv.y, cr, ai);
        }
    }
    if constexpr (kLdsRootsChained<MT>)
        pairs_chained_loop<MT, BIGC>(D, g, t1, r1, lane, n, sq, gp, ldc, ar, ai);
    else
        all_pairs_chained<MT, BIGC>(std::make_integer_sequence<int, P>{}, D, t1, r1, lane, n, R, gp,
                                    ldc, ar, ai);
    if (live) HC[g] = make_double2(ar, ai);
}

}  // namespace mc
