// H.C in the case-split form (tables in the reduced form, M <= 8).
//
// The two-body sum of Eq. (Haction) runs over removal pairs {k, s} and
// creation pairs {q, l}.  Where the two pairs coincide the configuration
// does not change; where they share one orbital the net effect is a single
// jump; only disjoint pairs move two particles (the coincident-index cases
// of the appendix on matrix elements).  Summing the amplitudes per target
// turns the first two groups into per-row coefficients of C_g and of the
// single-jump gathers that the one-body term already makes:
//
//   coincident:  A_ks B_ks = n_k n_s (k < s),  n_k (n_k - 1) (k = s)
//   one shared orbital c, net a -> b:  A_{ac} B_{cb} = (n_c - [c = a]) sqrt(n_a (n_b + 1))
//
// so the row coefficient is quadratic and the single-jump coefficient linear
// in the occupations, with constants staged once per call (k_prep_split).
// The disjoint pairs are gathered from the reduced double-jump map or, with
// no map, as two chained single jumps.  B_ql of a disjoint pair is taken on
// the row's own occupations, since q and l are untouched by the removal.
//
// Staged constants (complex), g' = staged pair coefficient incl. the 1/2:
//   DL[k]        h_kk - I_kk
//   GI[p]        I_ks = g'_{ks,ks} + g'_{ks,sk} (k < s), g'_{kk,kk}
//   HS[a*M+b]    h_ab - S_aba                      (a != b)
//   GS[(a*M+b)*M+c]  S_abc = g'_{ac,cb} + g'_{ac,bc} (c != b), g'_{ac,bb}
//   GD[pair p, slot r]  g'_{ks,ql} + g'_{ks,lq} (q < l), g'_{ks,qq}
#pragma once

#include <utility>

#include "mc_apply.h"

namespace mc {

// A wave-uniform true that the compiler cannot see through.  Branching on
// it puts each batch of a long straight-line stream into a basic block of its
// own; within one huge block the instruction scheduler issues every load of
// the stream first and keeps all gathered values live (hundreds of spilled
// registers), across blocks it cannot move them.
__device__ __forceinline__ bool opaque_true()
{
    int v;
    asm volatile("s_mov_b32 %0, 1" : "=s"(v));
    return v != 0;
}

// Rank of the creation pair (q, l), q <= l, among the pairs of orbitals
// outside {K, S}, in lexicographic order (closed form, so that it folds to a
// constant when its arguments are).
__host__ __device__ constexpr int reduced_rank(int M, int K, int S, int q, int l)
{
    const int E = M - (K == S ? 1 : 2);
    const int qq = q - (q > K) - (S != K && q > S);
    const int ll = l - (l > K) - (S != K && l > S);
    return qq * E - qq * (qq - 1) / 2 + (ll - qq);
}

// Whether slot (q, l), q <= l, of pair (K, S) is a true double jump.
__host__ __device__ constexpr bool reduced_slot(int K, int S, int q, int l)
{
    return q != K && q != S && l != K && l != S;
}

// Offset of pair p's constants within GD.
__host__ __device__ constexpr int reduced_pair_offset(int M, int p)
{
    int o = 0;
    for (int i = 0; i < p; ++i) o += reduced_slots(M, pair_k(M, i), pair_s(M, i));
    return o;
}

// Staged constants of the case-split apply from h and g (or their
// adjoints, g^dagger_ksql = conj(g_lqsk)): entries first, first + stride, ...
__device__ inline void stage_split_constants(int M, int adjoint, const double2 *__restrict__ g,
                                             const double2 *__restrict__ h,
                                             double2 *__restrict__ cf, int first, int stride)
{
    auto gat = [&](int k, int s, int q, int l) -> double2 {
        if (!adjoint) return g[((k * M + s) * M + q) * M + l];
        const double2 v = g[((l * M + q) * M + s) * M + k];
        return make_double2(v.x, -v.y);
    };
    auto add = [](double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); };
    auto sub = [](double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); };
    // g'_{ks,ql} for the unordered removal pair {k, s}
    auto gpv = [&](int k, int s, int q, int l) -> double2 {
        const int a = k < s ? k : s, b = k < s ? s : k;
        double2 v = gat(a, b, q, l);
        if (a != b) v = add(v, gat(b, a, q, l));
        return make_double2(0.5 * v.x, 0.5 * v.y);
    };
    auto hv = [&](int k, int l) -> double2 {
        const double2 v = adjoint ? h[l * M + k] : h[k * M + l];
        return make_double2(v.x, adjoint ? -v.y : v.y);
    };
    auto gi = [&](int k, int s) -> double2 {
        double2 v = gpv(k, s, k, s);
        if (k != s) v = add(v, gpv(k, s, s, k));
        return v;
    };
    auto gs = [&](int a, int b, int c) -> double2 {
        return c != b ? add(gpv(a, c, c, b), gpv(a, c, b, c)) : gpv(a, c, b, b);
    };
    const int total = split_total(M);
    for (int idx = first; idx < total; idx += stride) {
        double2 v = make_double2(0.0, 0.0);
        if (idx < split_gi_offset(M)) {
            const int k = idx;
            v = sub(hv(k, k), gi(k, k));
        } else if (idx < split_hs_offset(M)) {
            int p = idx - split_gi_offset(M), k = 0;
            while (p >= M - k) {
                p -= M - k;
                ++k;
            }
            v = gi(k, k + p);
        } else if (idx < split_gs_offset(M)) {
            const int j = idx - split_hs_offset(M), a = j / M, b = j % M;
            if (a != b) v = sub(hv(a, b), gs(a, b, a));
        } else if (idx < split_gd_offset(M)) {
            const int e = idx - split_gs_offset(M), j = e / M, c = e % M, a = j / M, b = j % M;
            if (a != b) v = gs(a, b, c);
        } else {
            // pair and reduced slot of entry e, both in lexicographic order
            int e = idx - split_gd_offset(M);
            int k = 0, s = 0;
            for (k = 0; k < M; ++k) {
                for (s = k; s < M; ++s) {
                    const int nd = reduced_slots(M, k, s);
                    if (e < nd) break;
                    e -= nd;
                }
                if (s < M) break;
            }
            for (int q = 0; q < M; ++q)
                for (int l = q; l < M; ++l) {
                    if (q == k || q == s || l == k || l == s) continue;
                    if (e-- == 0) v = q < l ? add(gpv(k, s, q, l), gpv(k, s, l, q)) : gpv(k, s, q, q);
                }
        }
        cf[idx] = v;
    }
}

// Contribution of removal pair P through the reduced map block at `pos`
// (nd(K, S) * 64 entries): A_KS sum_r GD[P][r] B_r C[t2r slot r].  All
// slot reads, then all gathers, then the arithmetic (nd <= 10 at M <= 5).
template <int MT, bool BIGC, int P>
__device__ __forceinline__ void split_pair_map(const int32_t *t2r, int64_t pos, int lane,
                                               const int (&n)[MT], const RowSq<MT> &R,
                                               const double2 *__restrict__ gd,
                                               const Gather<BIGC> &ldc, double &ar, double &ai)
{
    constexpr int K = pair_k(MT, P), S = pair_s(MT, P);
    constexpr int ND = reduced_slots(MT, K, S);
    constexpr int CO = reduced_pair_offset(MT, P);
    const bool valid = K == S ? n[K] >= 2 : (n[K] >= 1 && n[S] >= 1);
    const double A =
        valid ? R.template root<0>(K) * (K == S ? R.template root<-1>(K) : R.template root<0>(S))
              : 0.0;
    const __amdgpu_buffer_rsrc_t r2 = make_rsrc(t2r + pos, (uint32_t)(ND * kTile * 4));
    int32_t t[ND];
    double2 c[ND];
#pragma unroll
    for (int r = 0; r < ND; ++r) t[r] = buf_ld_i32(r2, (uint32_t)((r * kTile + lane) * 4), 0);
#pragma unroll
    for (int r = 0; r < ND; ++r) c[r] = ldc(t[r]);
    double br = 0.0, bi = 0.0;
#pragma unroll
    for (int j = 0; j < MT * MT; ++j) {
        const int q = j / MT, l = j % MT;
        if (l < q || !reduced_slot(K, S, q, l)) continue;
        const int r = reduced_rank(MT, K, S, q, l);
        const double Bf = q == l ? R.template root<1>(q) * R.template root<2>(q)
                                 : R.template root<1>(q) * R.template root<1>(l);
        const double cr = c[r].x * Bf, ci = c[r].y * Bf;
        const double2 Gv = gd[CO + r];
        br = fma(Gv.x, cr, br);
        br = fma(-Gv.y, ci, br);
        bi = fma(Gv.x, ci, bi);
        bi = fma(Gv.y, cr, bi);
    }
    ar = fma(A, br, ar);
    ai = fma(A, bi, ai);
}

template <int MT, bool BIGC, int... Ps>
__device__ __forceinline__ void split_pairs_map(std::integer_sequence<int, Ps...>,
                                                const uint64_t *pm, const int32_t *t2r,
                                                int64_t off0, int64_t off1, int lane,
                                                const int (&n)[MT], const RowSq<MT> &R,
                                                const double2 *__restrict__ gd,
                                                const Gather<BIGC> &ldc, double &ar, double &ai)
{
    int64_t pos = off0;
    (
        [&] {
            constexpr int NSB = reduced_slots(MT, pair_k(MT, Ps), pair_s(MT, Ps)) * kTile;
            if constexpr (NSB > 0) {
                if (((pm[Ps >> 6] >> (Ps & 63)) & 1) && pos + NSB <= off1) {
                    split_pair_map<MT, BIGC, Ps>(t2r, pos, lane, n, R, gd, ldc, ar, ai);
                    pos += NSB;
                }
            }
        }(),
        ...);
}

// Reduced slots of pair (K, S) among the ordered slots j = q*M + l in [J0, J1).
__host__ __device__ constexpr int reduced_in_range(int M, int K, int S, int J0, int J1)
{
    int c = 0;
    for (int j = J0; j < J1; ++j) {
        const int q = j / M, l = j % M;
        if (l >= q && reduced_slot(K, S, q, l)) ++c;
    }
    return c;
}

// Slots j in [J0, J1) of pair P through two chained single jumps, in a basic
// block of its own (gathers of one part in flight at a time).
template <int MT, bool BIGC, int P, int J0, int J1, bool OWN_BLOCK>
__device__ __forceinline__ void split_chain_part(int64_t D, const int32_t *__restrict__ t1,
                                                 int lane, const int32_t (&fh)[MT], bool valid,
                                                 const RowSq<MT> &R,
                                                 const double2 *__restrict__ gd,
                                                 const Gather<BIGC> &ldc, double &br, double &bi)
{
    constexpr int K = pair_k(MT, P), S = pair_s(MT, P), NS = MT * MT;
    constexpr int CO = reduced_pair_offset(MT, P);
    constexpr int NA = reduced_in_range(MT, K, S, J0, J1);
    constexpr int R0 = reduced_in_range(MT, K, S, 0, J0);
    if constexpr (NA > 0) {
        if constexpr (OWN_BLOCK)
            if (!opaque_true()) return;
        int32_t t[NA];
        double2 c[NA];
#pragma unroll
        for (int j = J0; j < J1; ++j) {
            const int q = j / MT, l = j % MT;
            if (l < q || !reduced_slot(K, S, q, l)) continue;
            const int r = reduced_rank(MT, K, S, q, l) - R0;
            const int32_t b = fh[q];
            const bool ok = valid && b >= 0 && b < D;
            const int64_t bb = ok ? b : 0;
            const int32_t v = t1[((bb >> 6) * NS + S * MT + l) * kTile + (bb & 63)];
            t[r] = ok ? v : -1;
        }
#pragma unroll
        for (int r = 0; r < NA; ++r) c[r] = ldc(t[r]);
#pragma unroll
        for (int j = J0; j < J1; ++j) {
            const int q = j / MT, l = j % MT;
            if (l < q || !reduced_slot(K, S, q, l)) continue;
            const int r = reduced_rank(MT, K, S, q, l);
            const double Bf = q == l ? R.template root<1>(q) * R.template root<2>(q)
                                     : R.template root<1>(q) * R.template root<1>(l);
            const double cr = c[r - R0].x * Bf, ci = c[r - R0].y * Bf;
            const double2 Gv = gd[CO + r];
            br = fma(Gv.x, cr, br);
            br = fma(-Gv.y, ci, br);
            bi = fma(Gv.x, ci, bi);
            bi = fma(Gv.y, cr, bi);
        }
    }
}

template <int MT, bool BIGC, int P, int... Hs>
__device__ __forceinline__ void split_chain_parts(std::integer_sequence<int, Hs...>, int64_t D,
                                                  const int32_t *__restrict__ t1, int lane,
                                                  const int32_t (&fh)[MT], bool valid,
                                                  const RowSq<MT> &R,
                                                  const double2 *__restrict__ gd,
                                                  const Gather<BIGC> &ldc, double &br, double &bi)
{
    constexpr int NS = MT * MT, NH = sizeof...(Hs);
    (split_chain_part<MT, BIGC, P, Hs * NS / NH, (Hs + 1) * NS / NH, (NH > 1)>(
         D, t1, lane, fh, valid, R, gd, ldc, br, bi),
     ...);
}

// The same pair through two chained single jumps: first K -> q from the
// tile's own single-jump block, then S -> l from the intermediate row; the
// slots in parts of at most 14 gathers.
template <int MT, bool BIGC, int P>
__device__ __forceinline__ void split_pair_chain(int64_t D, const int32_t *__restrict__ t1,
                                                 __amdgpu_buffer_rsrc_t r1, int lane,
                                                 const int (&n)[MT], const RowSq<MT> &R,
                                                 const double2 *__restrict__ gd,
                                                 const Gather<BIGC> &ldc, double &ar, double &ai)
{
    constexpr int K = pair_k(MT, P), S = pair_s(MT, P);
    constexpr int ND = reduced_slots(MT, K, S);
    if constexpr (ND > 0) {
        const bool valid = K == S ? n[K] >= 2 : (n[K] >= 1 && n[S] >= 1);
        if (!__ballot(valid)) return;   // no row of the tile can lose (K, S)
        const double A = valid ? R.template root<0>(K) *
                                     (K == S ? R.template root<-1>(K) : R.template root<0>(S))
                               : 0.0;
        int32_t fh[MT];
#pragma unroll
        for (int q = 0; q < MT; ++q)
            fh[q] = (q != K && q != S)
                        ? buf_ld_i32(r1, (uint32_t)(((K * MT + q) * kTile + lane) * 4), 0)
                        : -1;
        double br = 0.0, bi = 0.0;
        split_chain_parts<MT, BIGC, P>(std::make_integer_sequence<int, (ND + 13) / 14>{}, D, t1,
                                       lane, fh, valid, R, gd, ldc, br, bi);
        ar = fma(A, br, ar);
        ai = fma(A, bi, ai);
    }
}

template <int MT, bool BIGC, int... Ps>
__device__ __forceinline__ void split_pairs_chain(std::integer_sequence<int, Ps...>, int64_t D,
                                                  const int32_t *__restrict__ t1,
                                                  __amdgpu_buffer_rsrc_t r1, int lane,
                                                  const int (&n)[MT], const RowSq<MT> &R,
                                                  const double2 *__restrict__ gd,
                                                  const Gather<BIGC> &ldc, double &ar, double &ai)
{
    (split_pair_chain<MT, BIGC, Ps>(D, t1, r1, lane, n, R, gd, ldc, ar, ai), ...);
}

// ---------------------------------------------------------------------------
// Tiles whose pair mask has every pair (nearly all tiles of large spaces):
// the tile's single jumps and reduced-map blocks form one stream of
// U = M(M-1) + sum_p nd(p) slots with a compile-time layout, processed in
// batches of MC_FLAT_BATCH slots; the next batch's index loads are issued
// while the current batch's gathers are in flight.  Same arithmetic, in the
// same order, as the per-pair path.  The build default walks the same slots
// in class-major order instead (below), which gathers fewer coefficients and
// groups the terms differently (results agree to rounding).
// ---------------------------------------------------------------------------
#ifndef MC_FLAT_BATCH
#define MC_FLAT_BATCH 16
#endif

template <int MT>
struct FlatTile {
    static constexpr int NSING = MT * (MT - 1);
    static constexpr int NDBL =
        MT * reduced_slots(MT, 0, 0) + (MT * (MT - 1) / 2) * (MT >= 2 ? reduced_slots(MT, 0, 1) : 0);
    static constexpr int U = NSING + NDBL;
    static constexpr int SB = U < MC_FLAT_BATCH ? U : MC_FLAT_BATCH;
    static constexpr int NB = (U + SB - 1) / SB;
};

// double slot e (pair-major) -> pair and slot within the pair
__host__ __device__ constexpr int flat_pair(int M, int e)
{
    for (int p = 0; p < M * (M + 1) / 2; ++p) {
        const int nd = reduced_slots(M, pair_k(M, p), pair_s(M, p));
        if (e < nd) return p;
        e -= nd;
    }
    return -1;
}
__host__ __device__ constexpr int flat_slot(int M, int e)
{
    for (int p = 0; p < M * (M + 1) / 2; ++p) {
        const int nd = reduced_slots(M, pair_k(M, p), pair_s(M, p));
        if (e < nd) return e;
        e -= nd;
    }
    return -1;
}
// r-th creation pair (q, l) outside {K, S}: q (which = 0) or l (which = 1)
__host__ __device__ constexpr int reduced_ql(int M, int K, int S, int r, int which)
{
    for (int q = 0; q < M; ++q)
        for (int l = q; l < M; ++l) {
            if (!reduced_slot(K, S, q, l)) continue;
            if (r-- == 0) return which ? l : q;
        }
    return -1;
}

template <int MT, int U>
__device__ __forceinline__ int32_t flat_load(__amdgpu_buffer_rsrc_t r1, __amdgpu_buffer_rsrc_t r2,
                                             int lane)
{
    constexpr int NSING = FlatTile<MT>::NSING;
    if constexpr (U < NSING) {
        constexpr int a = U / (MT - 1), bb = U % (MT - 1), b = bb + (bb >= a);
        return buf_ld_i32(r1, (uint32_t)(((a * MT + b) * kTile + lane) * 4), 0);
    } else {
        return buf_ld_i32(r2, (uint32_t)(((U - NSING) * kTile + lane) * 4), 0);
    }
}

template <int MT, int U>
__device__ __forceinline__ void flat_fma(const double2 &c, const int (&n)[MT], const RowSq<MT> &R,
                                         const double (&x)[MT], const double2 *__restrict__ HS,
                                         const double2 *__restrict__ GS,
                                         const double2 *__restrict__ GD, double &br, double &bi,
                                         double &ar, double &ai)
{
    constexpr int NSING = FlatTile<MT>::NSING;
    if constexpr (U < NSING) {
        constexpr int a = U / (MT - 1), bb = U % (MT - 1), b = bb + (bb >= a), j = a * MT + b;
        double er = HS[j].x, ei = HS[j].y;
#pragma unroll
        for (int k = 0; k < MT; ++k) {
            er = fma(GS[j * MT + k].x, x[k], er);
            ei = fma(GS[j * MT + k].y, x[k], ei);
        }
        const double f = R.template root<0>(a) * R.template root<1>(b);
        er *= f;
        ei *= f;
        ar = fma(er, c.x, ar);
        ar = fma(-ei, c.y, ar);
        ai = fma(er, c.y, ai);
        ai = fma(ei, c.x, ai);
    } else {
        constexpr int e = U - NSING;
        constexpr int P = flat_pair(MT, e), r = flat_slot(MT, e);
        constexpr int K = pair_k(MT, P), S = pair_s(MT, P);
        constexpr int q = reduced_ql(MT, K, S, r, 0), l = reduced_ql(MT, K, S, r, 1);
        const double Bf = q == l ? R.template root<1>(q) * R.template root<2>(q)
                                 : R.template root<1>(q) * R.template root<1>(l);
        const double cr = c.x * Bf, ci = c.y * Bf;
        const double2 Gv = GD[e];
        br = fma(Gv.x, cr, br);
        br = fma(-Gv.y, ci, br);
        bi = fma(Gv.x, ci, bi);
        bi = fma(Gv.y, cr, bi);
        if constexpr (r == reduced_slots(MT, K, S) - 1) {
            // last slot of the pair: weight by A_KS as the per-pair path does
            const bool valid = K == S ? n[K] >= 2 : (n[K] >= 1 && n[S] >= 1);
            const double A = valid ? R.template root<0>(K) *
                                         (K == S ? R.template root<-1>(K) : R.template root<0>(S))
                                   : 0.0;
            ar = fma(A, br, ar);
            ai = fma(A, bi, ai);
            br = 0.0;
            bi = 0.0;
        }
    }
}

template <int MT, int U0, int... Is>
__device__ __forceinline__ void flat_loads(std::integer_sequence<int, Is...>,
                                           int32_t (&t)[FlatTile<MT>::SB],
                                           __amdgpu_buffer_rsrc_t r1, __amdgpu_buffer_rsrc_t r2,
                                           int lane)
{
    ((U0 + Is < FlatTile<MT>::U ? (void)(t[Is] = flat_load<MT, U0 + Is>(r1, r2, lane)) : (void)0),
     ...);
}

template <int MT, int U0, int... Is>
__device__ __forceinline__ void flat_fmas(std::integer_sequence<int, Is...>,
                                          const double2 (&c)[FlatTile<MT>::SB], const int (&n)[MT],
                                          const RowSq<MT> &R, const double (&x)[MT],
                                          const double2 *__restrict__ HS,
                                          const double2 *__restrict__ GS,
                                          const double2 *__restrict__ GD, double &br, double &bi,
                                          double &ar, double &ai)
{
    (
        [&] {
            if constexpr (U0 + Is < FlatTile<MT>::U)
                flat_fma<MT, U0 + Is>(c[Is], n, R, x, HS, GS, GD, br, bi, ar, ai);
        }(),
        ...);
}

// batch B: gathers for the indices in `cur`, then the next batch's index
// loads into `nxt`, then the arithmetic of batch B
template <int MT, bool BIGC, int B>
__device__ __forceinline__ void flat_batches(int32_t (&cur)[FlatTile<MT>::SB],
                                             int32_t (&nxt)[FlatTile<MT>::SB],
                                             __amdgpu_buffer_rsrc_t r1, __amdgpu_buffer_rsrc_t r2,
                                             int lane, const int (&n)[MT], const RowSq<MT> &R,
                                             const double (&x)[MT], const double2 *__restrict__ HS,
                                             const double2 *__restrict__ GS,
                                             const double2 *__restrict__ GD,
                                             const Gather<BIGC> &ldc, double &br, double &bi,
                                             double &ar, double &ai)
{
    constexpr int SB = FlatTile<MT>::SB, NB = FlatTile<MT>::NB, U = FlatTile<MT>::U;
    if constexpr (B < NB) {
        // each batch in a basic block of its own (see opaque_true)
        if (opaque_true()) {
            double2 c[SB];
#pragma unroll
            for (int i = 0; i < SB; ++i)
                if (B * SB + i < U) c[i] = ldc(cur[i]);
            if constexpr (B + 1 < NB)
                flat_loads<MT, (B + 1) * SB>(std::make_integer_sequence<int, SB>{}, nxt, r1, r2,
                                             lane);
            flat_fmas<MT, B * SB>(std::make_integer_sequence<int, SB>{}, c, n, R, x, HS, GS, GD, br,
                                  bi, ar, ai);
        }
        flat_batches<MT, BIGC, B + 1>(nxt, cur, r1, r2, lane, n, R, x, HS, GS, GD, ldc, br, bi, ar,
                                      ai);
    }
}

// ---------------------------------------------------------------------------
// Class-major stream: fewer coefficient gathers per tile.
//
// Consecutive rows of a run (indices that differ by one particle moved
// between orbitals 0 and 1) share the prefix sums S_1 .. S_{M-1} (mc_direct.h
// has the closed form of the index, in which only G_0(S_0) = S_0 + 1 moves
// along a run), so a jump that changes S_m by Delta_m reaches index
// g - Delta_0 + K, where K depends only on the run and on
// (Delta_1 .. Delta_{M-2}).  Jumps with equal (Delta_1 .. Delta_{M-2}) form a
// class; with s = Delta_0(anchor) - Delta_0(U), slot U's target at row g is
// its anchor's target at row g + s (same run) and equally the anchor's
// target at row g plus s.  So only the anchors' targets are read from the
// source; a member takes the anchor's value from lane i + s (DPP wave
// shifts) where lane i + s holds a row of the same run and the anchor is
// possible there, and is gathered at the anchor's own target plus s on the
// other lanes (run and tile edges).  The row's own coefficient anchors the
// class of jumps within orbitals {0, 1}.  M = 5: 130 slots, 54 anchors.
// ---------------------------------------------------------------------------

// Change of S_m when particles leave R1, R2 and enter A1, A2 (-1: none).
__host__ __device__ constexpr int prefix_delta(int m, int R1, int R2, int A1, int A2)
{
    return (A1 >= 0 && A1 <= m) + (A2 >= 0 && A2 <= m) - (R1 >= 0 && R1 <= m) -
           (R2 >= 0 && R2 <= m);
}

// Removed (R1, R2) and created (A1, A2) orbitals of slot U of the case-split
// flat stream (-1: none); U = -1 is the row itself.
template <int MT>
__host__ __device__ constexpr void flat_jump(int U, int &R1, int &R2, int &A1, int &A2)
{
    R1 = R2 = A1 = A2 = -1;
    if (U < 0) return;
    constexpr int NSING = MT * (MT - 1);
    if (U < NSING) {
        const int a = U / (MT - 1), bb = U % (MT - 1);
        R1 = a;
        A1 = bb + (bb >= a);
        return;
    }
    const int e = U - NSING, P = flat_pair(MT, e), r = flat_slot(MT, e);
    R1 = pair_k(MT, P);
    R2 = pair_s(MT, P);
    A1 = reduced_ql(MT, R1, R2, r, 0);
    A2 = reduced_ql(MT, R1, R2, r, 1);
}

#ifndef MC_CLASS_STREAM
#define MC_CLASS_STREAM 1
#endif
// largest orbital count whose full tiles take the class-major stream, per
// form (the paper form's slots grow as M^4: 786 at M = 6, 1414 at M = 7;
// the reduced form's stream at M = 7 measured slower than its per-pair path,
// at 205 VGPRs)
#ifndef MC_STREAM_MAX_M_REDUCED
#define MC_STREAM_MAX_M_REDUCED 6
#endif
#ifndef MC_STREAM_MAX_M_PAPER
#define MC_STREAM_MAX_M_PAPER 6
#endif
constexpr int kStreamMaxMReduced = MC_STREAM_MAX_M_REDUCED;
constexpr int kStreamMaxMPaper = MC_STREAM_MAX_M_PAPER;
#ifndef MC_CLASS_BATCH
#define MC_CLASS_BATCH 16
#endif

// Slot stream of a full tile.  Form 0: the case-split sum (single jumps,
// then the true double jumps of the reduced map).  Form 1: the paper's sum
// (single jumps, then every slot q*M + l of every removal pair, pair-major,
// as in the paper's double-jump map).
template <int MT, int FORM>
struct SlotForm;

template <int MT>
struct SlotForm<MT, 0> {
    static constexpr int U = FlatTile<MT>::U;
    static constexpr void jump(int u, int &R1, int &R2, int &A1, int &A2)
    {
        flat_jump<MT>(u, R1, R2, A1, A2);
    }
};

template <int MT>
struct SlotForm<MT, 1> {
    static constexpr int NSING = MT * (MT - 1);
    static constexpr int U = NSING + MT * (MT + 1) / 2 * MT * MT;
    static constexpr void jump(int u, int &R1, int &R2, int &A1, int &A2)
    {
        if (u < NSING) {
            flat_jump<MT>(u, R1, R2, A1, A2);
            return;
        }
        const int e = u - NSING, P = e / (MT * MT), j = e % (MT * MT);
        R1 = pair_k(MT, P);
        R2 = pair_s(MT, P);
        A1 = j / MT;
        A2 = j % MT;
    }
};

template <int MT, int FORM>
__host__ __device__ constexpr int slot_delta(int u, int m)
{
    int R1 = 0, R2 = 0, A1 = 0, A2 = 0;
    SlotForm<MT, FORM>::jump(u, R1, R2, A1, A2);
    return prefix_delta(m, R1, R2, A1, A2);
}

// The stream in class-major order.  Slots that reach the same configuration
// (the paper form has many: q <-> l, and slots sharing an orbital, which are
// single jumps) form one position; its leader is the first such slot, whose
// removals every other one's include, so the leader is possible wherever
// any of them is.  Position i: leader slot[i] (-1: the row itself), slots
// gslot[gstart[i] .. gstart[i+1]) for the arithmetic; its value is the
// anchor at position anc[i] read from lane + sh[i].  Batches of whole
// classes of at most MC_CLASS_BATCH positions (a larger class is cut into
// parts, each with an anchor of its own).
template <int MT, int FORM>
struct ClassPlan {
    static_assert(MT >= 1 && MT <= 7, "class-major stream for M <= 7");
    static constexpr int U = SlotForm<MT, FORM>::U;
    static constexpr int NS = U + 1;   // slots and the row itself
    static constexpr int NK = 15625;   // full keys: 5^(M-1) <= 15625
    int np = 0;
    int slot[NS] = {};
    int anc[NS] = {};
    int sh[NS] = {};
    int gstart[NS + 1] = {};
    int gslot[NS] = {};
    int nb = 0;
    int bstart[NS + 1] = {};
    int anchors = 0;

    constexpr ClassPlan()
    {
        // Delta_0, the class key (Delta_1 .. Delta_{M-2}) and the full key
        // (Delta_0 .. Delta_{M-2}) of each slot, base 5
        int d0[NS] = {}, ck[NS] = {}, fk[NS] = {};
        for (int v = -1; v < U; ++v) {
            d0[v + 1] = slot_delta<MT, FORM>(v, 0);
            int k = 0;
            for (int m = MT - 2; m >= 1; --m) k = 5 * k + slot_delta<MT, FORM>(v, m) + 2;
            ck[v + 1] = k;
            fk[v + 1] = 5 * k + d0[v + 1] + 2;
        }
        // groups of slots with one target, in slot order
        int gof_key[NK] = {}, lead[NS] = {}, gof[NS] = {}, ng = 0;
        for (int k = 0; k < NK; ++k) gof_key[k] = -1;
        for (int v = -1; v < U; ++v) {
            int &gk = gof_key[fk[v + 1]];
            if (gk < 0) {
                gk = ng;
                lead[ng] = v;
                ++ng;
            }
            gof[v + 1] = gk;
        }
        // classes of groups, cut into parts
        bool used[NS] = {};
        int posg[NS] = {}, cnt[NS] = {};
        int pos = 0;
        for (int a = 0; a < ng; ++a) {
            if (used[a]) continue;
            int first = pos, part = 0, lg = a;
            for (int b = a; b < ng; ++b) {
                if (used[b] || ck[lead[b] + 1] != ck[lead[a] + 1]) continue;
                if (part == MC_CLASS_BATCH) {
                    first = pos;
                    part = 0;
                    lg = b;
                }
                used[b] = true;
                slot[pos] = lead[b];
                anc[pos] = first;
                sh[pos] = d0[lead[lg] + 1] - d0[lead[b] + 1];
                if (pos == first && lead[b] >= 0) ++anchors;
                posg[b] = pos;
                ++pos;
                ++part;
            }
        }
        np = pos;
        // each position's slots, in slot order
        for (int v = -1; v < U; ++v) ++cnt[posg[gof[v + 1]]];
        gstart[0] = 0;
        for (int i = 0; i < np; ++i) gstart[i + 1] = gstart[i] + cnt[i];
        int fill[NS] = {};
        for (int v = -1; v < U; ++v) {
            const int i = posg[gof[v + 1]];
            gslot[gstart[i] + fill[i]++] = v;
        }
        // greedy batches of whole parts
        int start = 0;
        nb = 0;
        bstart[0] = 0;
        while (start < np) {
            int end = start;
            while (end < np) {
                int cend = end + 1;
                while (cend < np && anc[cend] == anc[end]) ++cend;
                if (end > start && cend - start > MC_CLASS_BATCH) break;
                end = cend;
            }
            bstart[++nb] = end;
            start = end;
        }
    }
};

template <int MT, int FORM>
constexpr ClassPlan<MT, FORM> kClassPlan{};

// x moved s lanes: lane i receives lane i + s (s > 0: wave_shl, s < 0:
// wave_shr, one lane per step); lanes with no source get `fill`.
template <int S>
__device__ __forceinline__ int32_t lane_shift_i32(int32_t x, int32_t fill)
{
    if constexpr (S == 0) return x;
    else if constexpr (S > 0)
        return lane_shift_i32<S - 1>(__builtin_amdgcn_update_dpp(fill, x, 0x130, 0xF, 0xF, false),
                                     fill);
    else
        return lane_shift_i32<S + 1>(__builtin_amdgcn_update_dpp(fill, x, 0x138, 0xF, 0xF, false),
                                     fill);
}

// x moved s lanes where the lanes with no source may take any value (DPP
// with bound control: they read 0, and no fill register is set up).
template <int S>
__device__ __forceinline__ int32_t lane_shift_any_i32(int32_t x)
{
    if constexpr (S == 0) return x;
    else if constexpr (S > 0)
        return lane_shift_any_i32<S - 1>(__builtin_amdgcn_mov_dpp(x, 0x130, 0xF, 0xF, true));
    else
        return lane_shift_any_i32<S + 1>(__builtin_amdgcn_mov_dpp(x, 0x138, 0xF, 0xF, true));
}

template <int S>
__device__ __forceinline__ double2 lane_shift_c128(double2 v)
{
    if constexpr (S == 0) {
        return v;
    } else {
        int32_t w[4];
        __builtin_memcpy(w, &v, 16);
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = lane_shift_any_i32<S>(w[k]);
        double2 r;
        __builtin_memcpy(&r, w, 16);
        return r;
    }
}

// Constants and arithmetic of one slot: a single jump adds
// sqrt(n_a (n_b+1)) [HS_ab + sum_c n_c GS_abc] C, a true double jump
// A_KS B_ql GD C (A folded per slot, as the slots of a pair are not
// adjacent).
template <int MT, int FORM>
struct ClassConsts;

template <int MT>
struct ClassConsts<MT, 0> {
    const double2 *__restrict__ HS;
    const double2 *__restrict__ GS;
    const double2 *__restrict__ GD;
    const double (&x)[MT];
};

// the paper form: h and the pair coefficients G'_{P, q*M+l}
template <int MT>
struct ClassConsts<MT, 1> {
    const double2 *__restrict__ h;
    const double2 *__restrict__ gp;
};


__device__ __forceinline__ void cmac(double er, double ei, const double2 &c, double &ar, double &ai)
{
    ar = fma(er, c.x, ar);
    ar = fma(-ei, c.y, ar);
    ai = fma(er, c.y, ai);
    ai = fma(ei, c.x, ai);
}

template <int MT, int FORM, int U>
__device__ __forceinline__ void class_fma(const double2 &c, const RowSq<MT> &R,
                                          const ClassConsts<MT, FORM> &k, double &ar, double &ai)
{
    constexpr int NSING = MT * (MT - 1);
    if constexpr (FORM == 1) {
        if constexpr (U < 0) {
            return;
        } else if constexpr (U < NSING) {
            // h_ab sqrt(n_a (n_b + 1)) C
            constexpr int a = U / (MT - 1), bb = U % (MT - 1), b = bb + (bb >= a), j = a * MT + b;
            const double f = R.template root<0>(a) * R.template root<1>(b);
            cmac(k.h[j].x * f, k.h[j].y * f, c, ar, ai);
        } else {
            // A_KS G'_{P,ql} B_ql(m) C with m = n - e_K - e_S; A is zero on
            // rows that cannot lose (K, S)
            constexpr int e = U - NSING, P = e / (MT * MT), j = e % (MT * MT);
            constexpr int q = j / MT, l = j % MT, K = pair_k(MT, P), S = pair_s(MT, P);
            constexpr int dq = (q == K) + (q == S), dl = (l == K) + (l == S);
            const double Bf = q == l ? R.template root<1 - dq>(q) * R.template root<2 - dq>(q)
                                     : R.template root<1 - dq>(q) * R.template root<1 - dl>(l);
            const double A = R.template root<0>(K) *
                             (K == S ? R.template root<-1>(K) : R.template root<0>(S));
            const double w = A * Bf;
            const double cr = c.x * w, ci = c.y * w;
            const double2 Gv = k.gp[P * MT * MT + j];
            ar = fma(Gv.x, cr, ar);
            ar = fma(-Gv.y, ci, ar);
            ai = fma(Gv.x, ci, ai);
            ai = fma(Gv.y, cr, ai);
        }
    } else if constexpr (U < 0) {
        return;   // the row itself: its term is added before the stream
    } else if constexpr (U < NSING) {
        constexpr int a = U / (MT - 1), bb = U % (MT - 1), b = bb + (bb >= a), j = a * MT + b;
        const double f = R.template root<0>(a) * R.template root<1>(b);
        double er = k.HS[j].x, ei = k.HS[j].y;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            er = fma(k.GS[j * MT + m].x, k.x[m], er);
            ei = fma(k.GS[j * MT + m].y, k.x[m], ei);
        }
        cmac(er * f, ei * f, c, ar, ai);
    } else {
        constexpr int P = flat_pair(MT, U - NSING), r = flat_slot(MT, U - NSING);
        constexpr int K = pair_k(MT, P), S = pair_s(MT, P);
        constexpr int q = reduced_ql(MT, K, S, r, 0), l = reduced_ql(MT, K, S, r, 1);
        const double Bf = q == l ? R.template root<1>(q) * R.template root<2>(q)
                                 : R.template root<1>(q) * R.template root<1>(l);
        const double A = R.template root<0>(K) *
                         (K == S ? R.template root<-1>(K) : R.template root<0>(S));
        const double w = A * Bf;
        const double cr = c.x * w, ci = c.y * w;
        const double2 Gv = k.GD[U - NSING];
        ar = fma(Gv.x, cr, ar);
        ar = fma(-Gv.y, ci, ar);
        ai = fma(Gv.x, ci, ai);
        ai = fma(Gv.y, cr, ai);
    }
}

// Whether slot U is a possible jump from occupations n (its removals are
// there); an impossible jump has a zero amplitude.
template <int MT, int FORM, int U>
__device__ __forceinline__ bool slot_valid(const int (&n)[MT])
{
    constexpr auto rem = [] {
        int R1 = 0, R2 = 0, A1 = 0, A2 = 0;
        SlotForm<MT, FORM>::jump(U, R1, R2, A1, A2);
        return std::pair<int, int>(R1, R2);
    }();
    constexpr int R1 = rem.first, R2 = rem.second;
    if constexpr (R1 < 0) return true;
    else if constexpr (R2 < 0) return n[R1] >= 1;
    else if constexpr (R1 == R2) return n[R1] >= 2;
    else return n[R1] >= 1 && n[R2] >= 1;
}

// Run of each lane's row: g + n_0 is the index of the run's last row (the
// index falls by one per particle moved from orbital 1 to 0 along a run), so
// two rows share a run exactly when their keys are equal; -1 on rows past
// the end.  `at[s + kMaxShift]` is the key of lane + s (-1 off the wave).
constexpr int kMaxShift = 4;

template <int MT>
struct RunKeys {
    const int (&n)[MT];
    int32_t key;
    int32_t at[2 * kMaxShift + 1];
};

template <int... Ss>
__device__ __forceinline__ void run_key_shifts(std::integer_sequence<int, Ss...>, int32_t key,
                                               int32_t (&at)[2 * kMaxShift + 1])
{
    ((at[Ss] = lane_shift_i32<Ss - kMaxShift>(key, -1)), ...);
}

// The arithmetic of every slot of position I, on its one value.
// Complex coefficient of paper-form slot U (U >= 0) on this row, added to
// (er, ei): the single jump's h_ab sqrt(n_a (n_b + 1)), or the double jump's
// A_KS B_ql(m) G'_{P,ql}.
template <int MT, int U>
__device__ __forceinline__ void paper_coef(const RowSq<MT> &R, const ClassConsts<MT, 1> &k,
                                           double &er, double &ei)
{
    constexpr int NSING = MT * (MT - 1);
    if constexpr (U < NSING) {
        constexpr int a = U / (MT - 1), bb = U % (MT - 1), b = bb + (bb >= a), j = a * MT + b;
        const double f = R.template root<0>(a) * R.template root<1>(b);
        er = fma(k.h[j].x, f, er);
        ei = fma(k.h[j].y, f, ei);
    } else {
        constexpr int e = U - NSING, P = e / (MT * MT), j = e % (MT * MT);
        constexpr int q = j / MT, l = j % MT, K = pair_k(MT, P), S = pair_s(MT, P);
        constexpr int dq = (q == K) + (q == S), dl = (l == K) + (l == S);
        const double Bf = q == l ? R.template root<1 - dq>(q) * R.template root<2 - dq>(q)
                                 : R.template root<1 - dq>(q) * R.template root<1 - dl>(l);
        const double A = R.template root<0>(K) *
                         (K == S ? R.template root<-1>(K) : R.template root<0>(S));
        const double w = A * Bf;
        const double2 Gv = k.gp[P * MT * MT + j];
        er = fma(Gv.x, w, er);
        ei = fma(Gv.y, w, ei);
    }
}

// The arithmetic of every slot of position I, on its one value.  Slots that
// share the value (the paper form's q <-> l and coincident slots) add their
// coefficients first and multiply the value once.
template <int MT, int FORM, int I, int... Js>
__device__ __forceinline__ void group_fma(std::integer_sequence<int, Js...>, const double2 &c,
                                          const RowSq<MT> &R, const ClassConsts<MT, FORM> &k,
                                          double &ar, double &ai)
{
    constexpr ClassPlan<MT, FORM> cp = kClassPlan<MT, FORM>;
    constexpr int n0 = cp.gstart[I];
    constexpr int ns = sizeof...(Js);
    if constexpr (FORM == 1 && ns > 1) {
        // the row itself (slot -1) carries no coefficient of its own
        constexpr int first = cp.gslot[n0] < 0 ? 1 : 0;
        if constexpr (ns - first > 1) {
            double er = 0.0, ei = 0.0;
            (
                [&] {
                    if constexpr (Js >= first) paper_coef<MT, cp.gslot[n0 + Js]>(R, k, er, ei);
                }(),
                ...);
            cmac(er, ei, c, ar, ai);
            return;
        }
    }
    (class_fma<MT, FORM, cp.gslot[n0 + Js]>(c, R, k, ar, ai), ...);
}

// Batch B of the class-major stream (positions [I0, I1)): `tix` holds the
// batch's anchor targets (from the source: table loads or closed form).
// A member's target is never loaded: on a lane whose row shares its run with
// the row s lanes on, and where the anchor is possible there, it is the
// anchor's target at lane + s, so the value moves by a DPP shift; elsewhere
// (run and tile edges) it is the anchor's target at the lane itself plus s,
// gathered.  Only where the anchor is impossible at the lane itself (rare)
// is the member's own target read from the source.  A member impossible at
// a lane has a zero amplitude there and takes any finite value.
template <int MT, int FORM, bool BIGC, int B, class Src, int... Is>
__device__ __forceinline__ void class_batch(std::integer_sequence<int, Is...>, const Src &src,
                                            const int32_t (&tix)[MC_CLASS_BATCH], int32_t own_t,
                                            double2 own_c, const RowSq<MT> &R,
                                            const RunKeys<MT> &rk,
                                            const ClassConsts<MT, FORM> &k,
                                            const Gather<BIGC> &ldc, double &ar, double &ai)
{
    constexpr ClassPlan<MT, FORM> cp = kClassPlan<MT, FORM>;
    constexpr int I0 = cp.bstart[B], I1 = cp.bstart[B + 1];
    double2 v[MC_CLASS_BATCH];
    // anchors: gather (the row itself: its own coefficient)
    (
        [&] {
            constexpr int i = I0 + Is;
            if constexpr (i < I1 && cp.anc[i] == i) {
                if constexpr (cp.slot[i] < 0) v[Is] = own_c;
                else v[Is] = ldc(tix[Is]);
            }
        }(),
        ...);
    // members: an edge gather where the shifted anchor does not serve
    bool edge[MC_CLASS_BATCH], own[MC_CLASS_BATCH];
    bool any_own = false;
    (
        [&] {
            constexpr int i = I0 + Is;
            if constexpr (i < I1 && cp.anc[i] != i) {
                constexpr int S = cp.sh[i];
                static_assert(S >= -kMaxShift && S <= kMaxShift, "anchor shift out of range");
                const int32_t ta = cp.slot[cp.anc[i]] < 0 ? own_t : tix[cp.anc[i] - I0];
                if constexpr (S == 0) {
                    // the anchor's own target: only an impossible anchor fails
                    edge[Is] = slot_valid<MT, FORM, cp.slot[i]>(rk.n) && ta < 0;
                } else {
                    // (off the wave the key test already makes the lane an edge)
                    const int32_t at = lane_shift_any_i32<S>(ta);
                    edge[Is] = slot_valid<MT, FORM, cp.slot[i]>(rk.n) &&
                               (rk.at[S + kMaxShift] != rk.key || at < 0);
                    v[Is] = ldc(edge[Is] && ta >= 0 ? ta + S : -1);
                }
                own[Is] = edge[Is] && ta < 0;
                any_own = any_own || own[Is];
            }
        }(),
        ...);
    (
        [&] {
            constexpr int i = I0 + Is;
            if constexpr (i < I1 && cp.anc[i] != i) {
                if constexpr (cp.sh[i] == 0) {
                    v[Is] = v[cp.anc[i] - I0];
                } else {
                    const double2 sv = lane_shift_c128<cp.sh[i]>(v[cp.anc[i] - I0]);
                    if (!edge[Is]) v[Is] = sv;
                }
            }
        }(),
        ...);
    // wave-uniform and rare: members whose anchor is impossible on the lane
    if (__builtin_amdgcn_readfirstlane(__ballot(any_own) != 0)) {
        (
            [&] {
                constexpr int i = I0 + Is;
                if constexpr (i < I1 && cp.anc[i] != i) {
                    if (own[Is]) v[Is] = ldc(src.template target<cp.slot[i]>());
                }
            }(),
            ...);
    }
    (
        [&] {
            constexpr int i = I0 + Is;
            if constexpr (i < I1)
                group_fma<MT, FORM, i>(
                    std::make_integer_sequence<int, cp.gstart[i + 1] - cp.gstart[i]>{}, v[Is], R,
                    k, ar, ai);
        }(),
        ...);
}

// Target index of the anchors of batch B from the source (the row itself
// needs none; members are derived).
template <int MT, int FORM, int B, class Src, int... Is>
__device__ __forceinline__ void class_targets(std::integer_sequence<int, Is...>, const Src &src,
                                              int32_t (&tix)[MC_CLASS_BATCH])
{
    constexpr ClassPlan<MT, FORM> cp = kClassPlan<MT, FORM>;
    constexpr int I0 = cp.bstart[B], I1 = cp.bstart[B + 1];
    (
        [&] {
            constexpr int i = I0 + Is;
            if constexpr (i < I1 && cp.slot[i] >= 0 && cp.anc[i] == i)
                tix[Is] = src.template target<cp.slot[i]>();
        }(),
        ...);
}

// The whole stream: batch B's block issues batch B+1's targets (table loads
// in flight during B's gathers), then B's gathers and arithmetic.
template <int MT, int FORM, bool BIGC, int B, class Src>
__device__ __forceinline__ void class_batches(int32_t (&cur)[MC_CLASS_BATCH],
                                              int32_t (&nxt)[MC_CLASS_BATCH], const Src &src,
                                              int32_t own_t, double2 own_c, const RowSq<MT> &R,
                                              const RunKeys<MT> &rk,
                                              const ClassConsts<MT, FORM> &k,
                                              const Gather<BIGC> &ldc, double &ar, double &ai)
{
    constexpr int NB = kClassPlan<MT, FORM>.nb;
    if constexpr (B < NB) {
        // each batch in a basic block of its own (see opaque_true)
        if (opaque_true()) {
            if constexpr (B + 1 < NB)
                class_targets<MT, FORM, B + 1>(std::make_integer_sequence<int, MC_CLASS_BATCH>{},
                                               src, nxt);
            class_batch<MT, FORM, BIGC, B>(std::make_integer_sequence<int, MC_CLASS_BATCH>{}, src,
                                           cur, own_t, own_c, R, rk, k, ldc, ar, ai);
        }
        class_batches<MT, FORM, BIGC, B + 1>(nxt, cur, src, own_t, own_c, R, rk, k, ldc, ar, ai);
    }
}

// `n`: the row's occupations; own_t: its index (negative past the end).
template <int MT, int FORM, bool BIGC, class Src>
__device__ __forceinline__ void class_stream(const Src &src, int32_t own_t, double2 own_c,
                                             const int (&n)[MT], const RowSq<MT> &R,
                                             const ClassConsts<MT, FORM> &k,
                                             const Gather<BIGC> &ldc, double &ar, double &ai)
{
    RunKeys<MT> rk{n, own_t >= 0 ? own_t + n[0] : -1, {}};
    run_key_shifts(std::make_integer_sequence<int, 2 * kMaxShift + 1>{}, rk.key, rk.at);
    int32_t ta[MC_CLASS_BATCH], tb[MC_CLASS_BATCH];
    class_targets<MT, FORM, 0>(std::make_integer_sequence<int, MC_CLASS_BATCH>{}, src, ta);
    class_batches<MT, FORM, BIGC, 0>(ta, tb, src, own_t, own_c, R, rk, k, ldc, ar, ai);
}

// Targets of a full tile through the tables: the tile's single-jump block
// and its double-jump block (every pair present, in order; form 0: the
// reduced map's true double jumps, form 1: the paper map's M*M slots per
// pair), column U - M(M-1) of the block either way.
template <int MT, int FORM>
struct MapSlots {
    __amdgpu_buffer_rsrc_t r1, r2;
    int lane;
    template <int U>
    __device__ __forceinline__ int32_t target() const
    {
        constexpr int NSING = MT * (MT - 1);
        if constexpr (U < NSING) {
            constexpr int a = U / (MT - 1), bb = U % (MT - 1), b = bb + (bb >= a);
            return buf_ld_i32(r1, (uint32_t)(((a * MT + b) * kTile + lane) * 4), 0);
        } else {
            return buf_ld_i32(r2, (uint32_t)(((U - NSING) * kTile + lane) * 4), 0);
        }
    }
};

// One 64-row tile of H.C in the case-split form; MAP: true double jumps from
// the reduced map, else chained.  `cf` holds the staged constants.
template <int MT, typename OccT, bool BIGC, bool MAP>
__device__ __forceinline__ void apply_tile_split(int64_t tile, int64_t D, int64_t cap,
                                                 const double *sq, const OccT *__restrict__ occ,
                                                 const int32_t *__restrict__ t1,
                                                 const uint64_t *__restrict__ pmask,
                                                 const int64_t *__restrict__ t2_off,
                                                 const int32_t *__restrict__ t2r,
                                                 const double2 *__restrict__ cf,
                                                 const double2 *__restrict__ C,
                                                 double2 *__restrict__ HC)
{
    constexpr int M = MT;
    constexpr int P = M * (M + 1) / 2;
    constexpr int W = (P + 63) / 64;
    constexpr int NS = M * M, SB = kSlotBatch<MT>;
    const int lane = threadIdx.x & 63;
    const int64_t g = tile * kTile + lane;
    const bool live = g < D;
    int n[M];
    RowSq<M> R;
    load_row<MT, OccT>(occ, tile, lane, n, R, sq);
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

    const __amdgpu_buffer_rsrc_t r1 = make_rsrc(t1 + tile * NS * kTile, (uint32_t)(NS * kTile * 4));
    if constexpr (MAP && MT <= kStreamMaxMReduced && FlatTile<MT>::NDBL > 0) {
        // every pair present and the block exactly the full size: one stream
        int64_t off0, off1;
        t2_block(t2_off, tile, cap, off0, off1);
        bool full = off1 - off0 == (int64_t)FlatTile<MT>::NDBL * kTile;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const int bits = P - 64 * w < 64 ? P - 64 * w : 64;
            const uint64_t want = bits == 64 ? ~(uint64_t)0 : (((uint64_t)1 << bits) - 1);
            full = full && pmask[tile * W + w] == want;
        }
        if (full) {
            const __amdgpu_buffer_rsrc_t r2 =
                make_rsrc(t2r + off0, (uint32_t)(FlatTile<MT>::NDBL * kTile * 4));
#if MC_CLASS_STREAM
            const MapSlots<MT, 0> src{r1, r2, lane};
            const ClassConsts<MT, 0> k{HS, GS, GD, x};
            class_stream<MT, 0, BIGC>(src, live ? (int32_t)g : -2, cg, n, R, k, ldc, ar, ai);
#else
            int32_t ta[FlatTile<MT>::SB], tb[FlatTile<MT>::SB];
            flat_loads<MT, 0>(std::make_integer_sequence<int, FlatTile<MT>::SB>{}, ta, r1, r2, lane);
            double br = 0.0, bi = 0.0;
            flat_batches<MT, BIGC, 0>(ta, tb, r1, r2, lane, n, R, x, HS, GS, GD, ldc, br, bi, ar, ai);
#endif
            if (live) HC[g] = make_double2(ar, ai);
            return;
        }
    }

    // single jumps a -> b with coefficient sqrt(n_a (n_b+1)) (HS + sum_c n_c GS)
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
            const int a = j / M, b = j % M;
            if (a == b) continue;
            double er = HS[j].x, ei = HS[j].y;
#pragma unroll
            for (int k = 0; k < M; ++k) {
                er = fma(GS[j * M + k].x, x[k], er);
                ei = fma(GS[j * M + k].y, x[k], ei);
            }
            const double f = R.template root<0>(a) * R.template root<1>(b);
            er *= f;
            ei *= f;
            ar = fma(er, c[i].x, ar);
            ar = fma(-ei, c[i].y, ar);
            ai = fma(er, c[i].y, ai);
            ai = fma(ei, c[i].x, ai);
        }
    }

    // true double jumps: a compile-time fold over the removal pairs, one
    // basic block per pair (chained pairs of more than 14 slots in parts of
    // their own), so every orbital index is a constant and nothing spills up
    // to M = 8
    if constexpr (MAP) {
        int64_t off0, off1;
        t2_block(t2_off, tile, cap, off0, off1);
        split_pairs_map<MT, BIGC>(std::make_integer_sequence<int, P>{}, pmask + tile * W, t2r, off0,
                                  off1, lane, n, R, GD, ldc, ar, ai);
    } else {
        split_pairs_chain<MT, BIGC>(std::make_integer_sequence<int, P>{}, D, t1, r1, lane, n, R, GD,
                                    ldc, ar, ai);
    }
    if (live) HC[g] = make_double2(ar, ai);
}

// One 64-row tile of H.C in the paper's form (the paper's double-jump map,
// M*M slots per removal pair).  A full tile (every removal pair present and
// its whole block in the map), for 2 <= M <= kStreamMaxMPaper, walks the class-major
// stream: the paper's sum over all its slots, reading only the anchors'
// table columns and gathering each distinct target once; other tiles take
// the per-pair path.
#ifndef MC_PAPER_STREAM
#define MC_PAPER_STREAM 1
#endif

template <int MT, typename OccT, bool BIGC>
__device__ __forceinline__ void apply_tile_paper(int64_t tile, int64_t D, int64_t cap,
                                                 const double *sq, const OccT *__restrict__ occ,
                                                 const int32_t *__restrict__ t1,
                                                 const uint64_t *__restrict__ pmask,
                                                 const int64_t *__restrict__ t2_off,
                                                 const int32_t *__restrict__ t2,
                                                 const double2 *__restrict__ h,
                                                 const double2 *__restrict__ gp,
                                                 const double2 *__restrict__ C,
                                                 double2 *__restrict__ HC)
{
    if constexpr (MC_PAPER_STREAM && MT >= 2 && MT <= kStreamMaxMPaper) {
        constexpr int P = MT * (MT + 1) / 2, W = (P + 63) / 64, NS = MT * MT;
        int64_t off0, off1;
        t2_block(t2_off, tile, cap, off0, off1);
        bool full = off1 - off0 == (int64_t)P * NS * kTile;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const int bits = P - 64 * w < 64 ? P - 64 * w : 64;
            const uint64_t want = bits == 64 ? ~(uint64_t)0 : (((uint64_t)1 << bits) - 1);
            full = full && pmask[tile * W + w] == want;
        }
        if (full) {
            const int lane = threadIdx.x & 63;
            const int64_t g = tile * kTile + lane;
            const bool live = g < D;
            int n[MT];
            RowSq<MT> R;
            load_row<MT, OccT>(occ, tile, lane, n, R, sq);
            const Gather<BIGC> ldc(C, D);
            const double2 cg = ldc(live ? (int32_t)g : -1);
            // diagonal one-body part: sum_k h_kk n_k C_g
            double dr = 0.0, di = 0.0;
#pragma unroll
            for (int k = 0; k < MT; ++k) {
                dr = fma(h[k * MT + k].x, (double)n[k], dr);
                di = fma(h[k * MT + k].y, (double)n[k], di);
            }
            double ar = dr * cg.x - di * cg.y, ai = dr * cg.y + di * cg.x;
            const MapSlots<MT, 1> src{
                make_rsrc(t1 + tile * NS * kTile, (uint32_t)(NS * kTile * 4)),
                make_rsrc(t2 + off0, (uint32_t)(P * NS * kTile * 4)), lane};
            const ClassConsts<MT, 1> k{h, gp};
            class_stream<MT, 1, BIGC>(src, live ? (int32_t)g : -2, cg, n, R, k, ldc, ar, ai);
            if (live) HC[g] = make_double2(ar, ai);
            return;
        }
    }
    apply_tile_t2<MT, OccT, BIGC>(tile, D, cap, sq, occ, t1, pmask, t2_off, t2, h, gp, C, HC);
}

}  // namespace mc
