// One- and two-body reduced density matrices (Eqs. rho1, rho2) as Gram
// matrices over the configurations of N-1 and N-2 particles.
//
// Moving the annihilators of Eqs. rho1 and rho2 onto the ket,
//
//   rho_kl   = < a_k Psi | a_l Psi >         = sum_m conj(X1_m[k])  X1_m[l],
//   rho_ksql = < a_s a_k Psi | a_q a_l Psi > = sum_m conj(X2_m[ks]) X2_m[ql],
//
// where m runs over the configurations of N-1 (resp. N-2) particles and
//
//   X1_m[l]  = (a_l Psi)_m     = sqrt(m_l + 1) C[m + e_l],
//   X2_m[ql] = (a_q a_l Psi)_m = sqrt((m_q + 1)(m_l + 1 + [q = l])) C[m + e_q + e_l]
//
// (bosonic ladder amplitudes, Sec. II; X2 is symmetric in q, l because the
// annihilators commute).  So rho1 is the M x M Gram matrix of the vectors
// X1_m, and rho2, indexed by unordered pairs {k,s}, {q,l}, the P x P Gram
// matrix of the X2_m, P = M(M+1)/2.  Each intermediate configuration costs
// P gathers, instead of one per (removal pair, creation slot) of every row;
// the symmetries rho_ksql = rho_skql = rho_kslq (commutation) and
// rho_ksql = conj(rho_qlks) (hermiticity) hold by construction, and only the
// upper triangle of the Gram matrix is accumulated.
//
// Where the targets m + e_q + e_l come from (the two sources below):
//  - no table: m is enumerated by its index in the space of N - L
//    particles; with S_j its prefix sums (mc_direct.h), those of
//    m + e_q + e_l are S_j + d_j, d_j = [q <= j] + [l <= j], so the target's
//    index is D_N - 1 - sum_{j=0}^{M-2} G_j(S_j + d_j), read from a per-row
//    table G_j(S_j + d), d = 0..L, with the compile-time d_j of each column
//    (S_j + d <= N keeps every G_j exact);
//  - the jump maps (Sec. IV): every m is reached exactly once from the row
//    gamma = m + L e_0 of the N-particle space (rows with n_0 >= L), whose
//    single jumps out of orbital 0 and double jumps out of the pair (0, 0)
//    are exactly m + e_l and m + e_q + e_l: T1[gamma][0][l] and the (0, 0)
//    block of the double-jump map (paper form: slot q M + l; reduced form:
//    the slots with q, l >= 1, the others being gamma itself and
//    T1[gamma][0][l]; without a map, two chained single jumps
//    T1[T1[gamma][0][q]][0][l]).
//
// Kernel.  One wavefront per block walks chunks of 64 intermediate
// configurations (lane = configuration): it computes its row of X into LDS,
// then the upper triangle of the chunk's Gram matrix is accumulated in
// BS x BS complex register blocks (BS of 2, 3 or 4: the least padding), one
// block pair (bi <= bj) per lane and the 64 rows split over 64 / #blocks lane
// groups.  The groups are summed in a fixed
// order at the end; partials per wavefront go to the workspace and are summed
// over wavefronts by a fixed tree: results are bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "mc.h"
#include "mc_direct.h"
#include "mc_internal.h"

namespace mc {

// Column layout of the lift of L particles (L = 1: one column per orbital;
// L = 2: one per unordered pair, lexicographic).
// Register block size of the Gram accumulation: of 2, 3 and 4, the one that
// pads the upper triangle least with at most 64 block pairs (one per lane).
__host__ __device__ constexpr int gram_block(int P)
{
    int best = 4, best_pad = 1 << 30;
    for (int bs = 2; bs <= 4; ++bs) {
        const int pb = (P + bs - 1) / bs, nb = pb * (pb + 1) / 2;
        if (nb > 64) continue;
        const int pad = nb * bs * bs;
        if (pad < best_pad) {
            best = bs;
            best_pad = pad;
        }
    }
    return best;
}

template <int MT, int L>
struct Lift {
    static constexpr int P = L == 1 ? MT : MT * (MT + 1) / 2;   // columns
    static constexpr int BS = gram_block(P);                     // register block size
    static constexpr int PB = (P + BS - 1) / BS;                  // column blocks
    static constexpr int PP = BS * PB;                            // padded columns
    static constexpr int NB = PB * (PB + 1) / 2;                  // block pairs bi <= bj
    static constexpr int R = 64 / NB;                             // lane groups over rows
    static constexpr int E = NB * BS * BS;                        // partial entries per wave
    static constexpr int STRIDE = PP + 1;                         // LDS row stride (double2)
    static constexpr int LDS = (64 * STRIDE > 64 * 16 ? 64 * STRIDE : 64 * 16) * 16;   // bytes
};

template <int MT, int L, int c>
__host__ __device__ constexpr int col_q() { return L == 1 ? c : pair_k(MT, c); }
template <int MT, int L, int c>
__host__ __device__ constexpr int col_l() { return L == 1 ? -1 : pair_s(MT, c); }

// Ladder amplitude of column (q, l) (l < 0: one particle) on occupations m.
template <int MT, int q, int l>
__device__ __forceinline__ double lift_amp(const int (&m)[MT])
{
    const double a = (double)m[q] + 1.0;
    if constexpr (l < 0) return sqrt(a);
    else if constexpr (q == l) return sqrt(a * (a + 1.0));
    else return sqrt(a * ((double)m[l] + 1.0));
}

constexpr int kGramBatch = 12;   // gathers per basic block

// Gathers of one batch of columns [C0, C0 + kGramBatch): target(c) gives the
// index (-1: none), the values amp * C[index] go to xrow[c].
template <int MT, int L, bool BIGC, int C0, class Tgt, int... Is>
__device__ __forceinline__ void gram_batch(std::integer_sequence<int, Is...>, const Tgt &tgt,
                                           const int (&m)[MT], const Gather<BIGC> &ldc,
                                           double2 *xrow)
{
    constexpr int P = Lift<MT, L>::P;
    int32_t t[sizeof...(Is)];
    double2 v[sizeof...(Is)];
    (
        [&] {
            constexpr int c = C0 + Is;
            if constexpr (c < P) t[Is] = tgt.template target<col_q<MT, L, c>(), col_l<MT, L, c>()>();
        }(),
        ...);
    (
        [&] {
            if constexpr (C0 + Is < P) v[Is] = ldc(t[Is]);
        }(),
        ...);
    (
        [&] {
            constexpr int c = C0 + Is;
            if constexpr (c < P) {
                const double a = lift_amp<MT, col_q<MT, L, c>(), col_l<MT, L, c>()>(m);
                xrow[c] = make_double2(a * v[Is].x, a * v[Is].y);
            }
        }(),
        ...);
}

template <int MT, int L, bool BIGC, class Tgt, int... Bs>
__device__ __forceinline__ void gram_row(std::integer_sequence<int, Bs...>, const Tgt &tgt,
                                         const int (&m)[MT], const Gather<BIGC> &ldc,
                                         double2 *xrow)
{
    (
        [&] {
            // each batch in a basic block of its own (see opaque_true)
            if (opaque_true())
                gram_batch<MT, L, BIGC, Bs * kGramBatch>(
                    std::make_integer_sequence<int, kGramBatch>{}, tgt, m, ldc, xrow);
        }(),
        ...);
}

template <int MT, int L>
constexpr int kGramBatches = (Lift<MT, L>::P + kGramBatch - 1) / kGramBatch;

// ---------------------------------------------------------------------------
// Source 1, no table: intermediate m by its index in the (N - L)-particle
// space; targets from the closed form.
// ---------------------------------------------------------------------------
template <int MT, int L>
struct LiftTargets {
    static constexpr int NE = MT > 1 ? MT - 1 : 1;
    bool live;
    uint32_t base;   // D_N - 1
    uint32_t G[NE][L + 1];

    template <int q, int l, int... Js>
    __device__ __forceinline__ uint32_t fold(std::integer_sequence<int, Js...>) const
    {
        return (base - ... - G[Js][(q <= Js) + (l >= 0 && l <= Js)]);
    }

    template <int q, int l>
    __device__ __forceinline__ int32_t target() const
    {
        return live ? (int32_t)fold<q, l>(std::make_integer_sequence<int, MT - 1>{}) : -1;
    }
};

template <int MT, int L, bool BIGC>
struct DirectSource {
    using Tgt = LiftTargets<MT, L>;
    int Nl, nbits;      // N - L and its bit width
    int64_t Dl, DN;     // dimensions of the N - L and N particle spaces

    // targets and occupations of intermediate configuration ch * 64 + lane
    __device__ __forceinline__ bool prepare(int64_t ch, int lane, Tgt &tg, int (&m)[MT]) const
    {
        const int64_t row = ch * 64 + lane;
        tg.live = row < Dl;
        int S[MT];
        direct_prefix<MT>(tg.live ? row : Dl - 1, Dl, Nl, nbits, S);
        m[0] = S[0];
#pragma unroll
        for (int j = 1; j < MT; ++j) m[j] = S[j] - S[j - 1];
        tg.base = (uint32_t)(DN - 1);
#pragma unroll
        for (int j = 0; j + 1 < MT; ++j)
#pragma unroll
            for (int d = 0; d <= L; ++d)
                tg.G[j][d] =
                    j == 0 ? (uint32_t)(S[0] + d) : (uint32_t)direct_g(j, (double)(S[j] + d));
        return true;
    }

    // the lane's row of X
    __device__ __forceinline__ bool fill(int64_t ch, int lane, const Gather<BIGC> &ldc,
                                         double2 *xrow) const
    {
        Tgt tg;
        int m[MT];
        prepare(ch, lane, tg, m);
        gram_row<MT, L, BIGC>(std::make_integer_sequence<int, kGramBatches<MT, L>>{}, tg, m, ldc,
                              xrow);
        return true;
    }
};

// ---------------------------------------------------------------------------
// Source 2, the jump maps: row gamma = m + L e_0 (n_0 >= L) of tile ch.
// KIND: 0 = no double-jump map (chained single jumps), 1 = paper form,
// 2 = reduced form.
// ---------------------------------------------------------------------------
template <int MT, int L, int KIND>
struct MapTargets {
    bool live;
    int32_t g;
    int32_t s0[MT];                         // T1[gamma][0][l]
    __amdgpu_buffer_rsrc_t r2;              // the tile's (0, 0) block (map kinds)
    const int32_t *__restrict__ t1;         // whole single-jump map (chained kind)
    int lane;

    __device__ __forceinline__ int32_t chain(int32_t u, int l) const
    {
        // T1[u][0][l]: tile u / 64, lane u % 64 (u >= 0 on live rows)
        const int64_t uu = u < 0 ? 0 : u;
        const int32_t v = t1[((uu >> 6) * (MT * MT) + l) * kTile + (uu & 63)];
        return u < 0 ? -1 : v;
    }

    template <int q, int l>
    __device__ __forceinline__ int32_t target() const
    {
        if (!live) return -1;
        if constexpr (l < 0) {
            return s0[q];   // one particle: m + e_q = T1[gamma][0][q]
        } else if constexpr (q == 0 && l == 0) {
            return g;
        } else if constexpr (q == 0) {
            return s0[l];
        } else if constexpr (KIND == 1) {
            return buf_ld_i32(r2, (uint32_t)(((q * MT + l) * kTile + lane) * 4), 0);
        } else if constexpr (KIND == 2) {
            return buf_ld_i32(r2, (uint32_t)((reduced_rank(MT, 0, 0, q, l) * kTile + lane) * 4), 0);
        } else {
            return chain(s0[q], l);
        }
    }
};

template <int MT, int L, typename OccT, int KIND, bool BIGC>
struct MapSource {
    using Tgt = MapTargets<MT, L, KIND>;
    int64_t D, cap;   // rows; capacity of the double-jump map (entries)
    const OccT *__restrict__ occ;
    const int32_t *__restrict__ t1;
    const uint64_t *__restrict__ pmask;
    const int64_t *__restrict__ t2_off;
    const int32_t *__restrict__ t2;

    // targets and occupations of the rows of tile `tile` (false: no row of
    // the tile has L particles in orbital 0; wave-uniform)
    __device__ __forceinline__ bool prepare(int64_t tile, int lane, Tgt &tg, int (&m)[MT]) const
    {
        constexpr int NS = MT * MT;
        tg.lane = lane;
        tg.t1 = t1;
        const int64_t g = tile * kTile + lane;
        int n[MT];
#pragma unroll
        for (int k = 0; k < MT; ++k) n[k] = (int)occ[(tile * MT + k) * kTile + lane];
        tg.live = g < D && n[0] >= L;
        tg.g = (int32_t)g;
        // occupations of m = n - L e_0 (zero on rows without one: their
        // amplitudes must stay finite, their values are zero)
#pragma unroll
        for (int k = 0; k < MT; ++k) m[k] = tg.live ? n[k] - (k == 0 ? L : 0) : 0;
        const __amdgpu_buffer_rsrc_t r1 = make_rsrc(t1 + tile * NS * kTile, (uint32_t)(NS * kTile * 4));
#pragma unroll
        for (int l = 0; l < MT; ++l)
            tg.s0[l] = l == 0 ? (int32_t)g : buf_ld_i32(r1, (uint32_t)((l * kTile + lane) * 4), 0);
        if constexpr (L == 2 && KIND != 0) {
            // pair (0, 0) is the first block of the tile when present
            constexpr int BS = KIND == 1 ? NS : MT * (MT - 1) / 2;
            const bool has = (pmask[tile * ((MT * (MT + 1) / 2 + 63) / 64)] & 1) != 0;
            int64_t off0, off1;
            t2_block(t2_off, tile, cap, off0, off1);
            const bool fits = has && off0 + (int64_t)BS * kTile <= off1;
            tg.r2 = make_rsrc(t2 + (fits ? off0 : 0), fits ? (uint32_t)(BS * kTile * 4) : 0u);
            if (!fits) tg.live = false;
        }
        return __builtin_amdgcn_readfirstlane(__ballot(tg.live) != 0);
    }

    __device__ __forceinline__ bool fill(int64_t tile, int lane, const Gather<BIGC> &ldc,
                                         double2 *xrow) const
    {
        Tgt tg;
        int m[MT];
        if (!prepare(tile, lane, tg, m)) return false;
        gram_row<MT, L, BIGC>(std::make_integer_sequence<int, kGramBatches<MT, L>>{}, tg, m, ldc,
                              xrow);
        return true;
    }
};

// Prefetch form of a row of X: every column's gather issued at once (values
// in registers), and later the amplitudes applied into LDS.
template <int MT, int L, bool BIGC, class Tgt, int... Cs>
__device__ __forceinline__ void gram_issue(std::integer_sequence<int, Cs...>, const Tgt &tgt,
                                           const Gather<BIGC> &ldc,
                                           double2 (&v)[Lift<MT, L>::P])
{
    int32_t t[sizeof...(Cs)];
    ((t[Cs] = tgt.template target<col_q<MT, L, Cs>(), col_l<MT, L, Cs>()>()), ...);
    ((v[Cs] = ldc(t[Cs])), ...);
}

template <int MT, int L, int... Cs>
__device__ __forceinline__ void gram_commit(std::integer_sequence<int, Cs...>, const int (&m)[MT],
                                            const double2 (&v)[Lift<MT, L>::P], double2 *xrow)
{
    (
        [&] {
            const double a = lift_amp<MT, col_q<MT, L, Cs>(), col_l<MT, L, Cs>()>(m);
            xrow[Cs] = make_double2(a * v[Cs].x, a * v[Cs].y);
        }(),
        ...);
}

// Up to this many columns the next chunk's gathers are kept in registers
// while the current chunk's Gram matrix is accumulated.
#ifndef MC_GRAM_PREFETCH_MAX_P
#define MC_GRAM_PREFETCH_MAX_P 21
#endif

// ---------------------------------------------------------------------------
// The Gram kernel over any source.
// ---------------------------------------------------------------------------
template <int MT, int L, bool BIGC, class Src>
__global__ __launch_bounds__(64) void k_gram(Src src, int64_t DN, int64_t chunks, int nwaves,
                                             const double2 *__restrict__ C,
                                             double2 *__restrict__ part)
{
    using LF = Lift<MT, L>;
    extern __shared__ double2 X[];   // [64][STRIDE]; reused for the group sums
    const int lane = threadIdx.x;
    const int wave = blockIdx.x;
#pragma unroll
    for (int c = LF::P; c < LF::PP; ++c) X[lane * LF::STRIDE + c] = make_double2(0.0, 0.0);
    // this lane's block pair (bi <= bj) and row group
    const int blk = lane % LF::NB, grp = lane / LF::NB;
    int bi = 0, rem = blk;
    while (rem >= LF::PB - bi) {
        rem -= LF::PB - bi;
        ++bi;
    }
    const int bj = bi + rem;
    constexpr int BS = LF::BS;
    double ar[BS][BS], ai[BS][BS];
#pragma unroll
    for (int i = 0; i < BS; ++i)
#pragma unroll
        for (int j = 0; j < BS; ++j) ar[i][j] = ai[i][j] = 0.0;
    const Gather<BIGC> ldc(C, DN);
    constexpr bool PRE = LF::P <= MC_GRAM_PREFETCH_MAX_P;
    typename Src::Tgt tg;
    int m[MT];
    double2 pv[PRE ? LF::P : 1];
    if constexpr (PRE) {
        if (wave < chunks) {
            src.prepare(wave, lane, tg, m);
            gram_issue<MT, L, BIGC>(std::make_integer_sequence<int, LF::P>{}, tg, ldc, pv);
        }
    }
    for (int64_t ch = wave; ch < chunks; ch += nwaves) {
        if constexpr (PRE) {
            // this chunk's values (in flight since the last chunk) into LDS,
            // then the next chunk's gathers, in flight during the arithmetic
            gram_commit<MT, L>(std::make_integer_sequence<int, LF::P>{}, m, pv,
                               X + lane * LF::STRIDE);
            __syncthreads();
            if (ch + nwaves < chunks) {
                src.prepare(ch + nwaves, lane, tg, m);
                gram_issue<MT, L, BIGC>(std::make_integer_sequence<int, LF::P>{}, tg, ldc, pv);
            }
        } else {
            // a chunk with no intermediate configuration adds nothing (wave-uniform)
            if (!src.fill(ch, lane, ldc, X + lane * LF::STRIDE)) continue;
            __syncthreads();
        }
        if (grp < LF::R) {
            for (int r = grp; r < 64; r += LF::R) {
                const double2 *xr = X + r * LF::STRIDE;
                double2 a[BS], b[BS];
#pragma unroll
                for (int i = 0; i < BS; ++i) {
                    a[i] = xr[BS * bi + i];
                    b[i] = xr[BS * bj + i];
                }
#pragma unroll
                for (int i = 0; i < BS; ++i)
#pragma unroll
                    for (int j = 0; j < BS; ++j) {
                        // conj(a_i) b_j
                        ar[i][j] = fma(a[i].x, b[j].x, fma(a[i].y, b[j].y, ar[i][j]));
                        ai[i][j] = fma(a[i].x, b[j].y, fma(-a[i].y, b[j].x, ai[i][j]));
                    }
            }
        }
        __syncthreads();
    }
    // sum the lane groups of each block pair in group order
    if (grp < LF::R) {
#pragma unroll
        for (int i = 0; i < BS; ++i)
#pragma unroll
            for (int j = 0; j < BS; ++j)
                X[(grp * LF::NB + blk) * BS * BS + i * BS + j] = make_double2(ar[i][j], ai[i][j]);
    }
    __syncthreads();
    for (int e = lane; e < LF::E; e += 64) {
        double sr = 0.0, si = 0.0;
        for (int g = 0; g < LF::R; ++g) {
            const double2 v = X[g * LF::E + e];
            sr += v.x;
            si += v.y;
        }
        part[(int64_t)e * nwaves + wave] = make_double2(sr, si);
    }
}

namespace {

// canon[e] = sum over waves of part[e][w]: a fixed strided split over 256
// threads and a fixed tree.
__global__ __launch_bounds__(256) void k_gram_sum(int nwaves, const double2 *__restrict__ part,
                                                  double2 *__restrict__ canon)
{
    __shared__ double sr[256], si[256];
    const int e = blockIdx.x, t = threadIdx.x;
    double r = 0.0, i = 0.0;
    for (int w = t; w < nwaves; w += 256) {
        const double2 v = part[(int64_t)e * nwaves + w];
        r += v.x;
        i += v.y;
    }
    sr[t] = r;
    si[t] = i;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            sr[t] += sr[t + s];
            si[t] += si[t + s];
        }
        __syncthreads();
    }
    if (t == 0) canon[e] = make_double2(sr[0], si[0]);
}

__device__ __forceinline__ int upair(int M, int x, int y)
{
    const int a = x < y ? x : y, b = x < y ? y : x;
    return a * M - a * (a - 1) / 2 + (b - a);
}

// The output from the canonical (column c1 <= c2) entries: rho1[k][l] is
// Gram entry (k, l); rho2[k][s][q][l] is entry ({k,s}, {q,l}).  Entries
// below the diagonal are conjugates, diagonal entries are real.  canon =
// NULL writes zeros (fewer than L particles).
__global__ __launch_bounds__(256) void k_gram_expand(int M, int L, int PB, int BS,
                                                     const double2 *__restrict__ canon,
                                                     double2 *__restrict__ out)
{
    const int total = L == 1 ? M * M : M * M * M * M;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    if (!canon) {
        out[idx] = make_double2(0.0, 0.0);
        return;
    }
    int c1, c2;
    if (L == 1) {
        c1 = idx / M;
        c2 = idx % M;
    } else {
        const int l = idx % M, q = (idx / M) % M, s = (idx / (M * M)) % M, k = idx / (M * M * M);
        c1 = upair(M, k, s);
        c2 = upair(M, q, l);
    }
    const bool swap = c1 > c2;
    const int x = swap ? c2 : c1, y = swap ? c1 : c2;
    const int bi = x / BS, bj = y / BS;
    const int blk = bi * PB - bi * (bi - 1) / 2 + (bj - bi);
    double2 v = canon[blk * BS * BS + (x % BS) * BS + (y % BS)];
    if (swap) v.y = -v.y;
    if (x == y) v.y = 0.0;
    out[idx] = v;
}

constexpr int64_t kGramMaxWaves = 2048;

// Shape of one call: wavefronts (from the LDS footprint: the resident
// wavefronts of 256 CUs, at most 8 per CU, fixed per (N, M) so results are
// reproducible on any device), partial entries, workspace bytes.
struct GramShape {
    int64_t chunks = 0, nwaves = 0, E = 0, PB = 0, BS = 0;
    size_t lds = 0, ws = 0;
};

template <int MT, int L>
void gram_shape_t(int64_t chunks, GramShape *g)
{
    int64_t per_cu = (160 * 1024) / Lift<MT, L>::LDS;
    per_cu = per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu);
    int64_t w = 256 * per_cu;
    w = w < kGramMaxWaves ? w : kGramMaxWaves;
    g->chunks = chunks;
    g->nwaves = chunks < w ? (chunks > 0 ? chunks : 1) : w;
    g->E = Lift<MT, L>::E;
    g->PB = Lift<MT, L>::PB;
    g->BS = Lift<MT, L>::BS;
    g->lds = Lift<MT, L>::LDS;
    g->ws = (size_t)(g->E * g->nwaves + g->E) * 16;
}

inline int gram_shape(int M, int L, int64_t chunks, GramShape *g)
{
    if (M < 1 || M > 8 || (L != 1 && L != 2)) return MC_EINVAL;
    MC_DISPATCH_M(M, if constexpr (MT > 0 && MT <= 8) {
        if (L == 1) (gram_shape_t<MT, 1>)(chunks, g);
        else (gram_shape_t<MT, 2>)(chunks, g);
    });
    return MC_OK;
}

// Zero output (fewer than L particles).
inline int gram_zero(int M, int L, double *out_d, hipStream_t s)
{
    const int total = L == 1 ? M * M : M * M * M * M;
    hipLaunchKernelGGL(k_gram_expand, dim3((total + 255) / 256), dim3(256), 0, s, M, L, 1, 1,
                       (const double2 *)nullptr, (double2 *)out_d);
    return launch_status();
}

// Launches the Gram kernel over `src`, the wave sum and the expansion.
template <int MT, int L, bool BIGC, class Src>
int gram_launch(const Src &src, int64_t DN, const GramShape &gs, const double *C_d,
                double *out_d, void *ws_d, hipStream_t s)
{
    double2 *part = (double2 *)ws_d;
    double2 *canon = part + gs.E * gs.nwaves;
    const int total = L == 1 ? MT * MT : MT * MT * MT * MT;
    hipLaunchKernelGGL((k_gram<MT, L, BIGC, Src>), dim3((unsigned)gs.nwaves), dim3(64), gs.lds, s,
                       src, DN, gs.chunks, (int)gs.nwaves, (const double2 *)C_d, part);
    hipLaunchKernelGGL(k_gram_sum, dim3((unsigned)gs.E), dim3(256), 0, s, (int)gs.nwaves, part,
                       canon);
    hipLaunchKernelGGL(k_gram_expand, dim3((total + 255) / 256), dim3(256), 0, s, MT, L,
                       (int)gs.PB, (int)gs.BS, (const double2 *)canon, (double2 *)out_d);
    return launch_status();
}

}  // namespace
}  // namespace mc
