// One- and two-body reduced density matrices (Eqs. rho1, rho2) with no
// table: each row's occupations and the configuration each pair of ladder
// operators leads to come from the row index in closed form (mc_direct.h).
//
//   rho1_kl   = sum_g conj(C_g) sqrt(n_k (n_l+1)) C[g - e_k + e_l]      (k != l)
//   rho1_kk   = sum_g |C_g|^2 n_k
//   rho2_ksql = sum_g conj(C_g) A_ks(n) B_ql(n - e_k - e_s) C[g - e_k - e_s + e_q + e_l]
//
// with A, B the amplitudes of mc_apply_H.  The closed-form target covers the
// coincident-index slots too: a creation into a removed orbital cancels in
// the prefix sums, so {q,l} = {k,s} gives the row itself and one shared
// orbital a single jump, with no case analysis.  rho2 is accumulated for
// unordered removal pairs (k <= s) and unordered creation pairs (q <= l) and
// expanded with rho2_ksql = rho2_skql = rho2_kslq (a+_k a+_s and a_q a_l
// commute; target and amplitudes are symmetric in each pair).
//
// Wave w accumulates tiles w, w + W, ... per slot in registers (chunks of
// kDRhoChunk slots per pass over the tiles), sums each slot over its 64 rows
// with a butterfly and leaves one partial per wave in the workspace; the
// partials are summed over waves in a fixed order, so results are bitwise
// reproducible.
#include <hip/hip_runtime.h>

#include <utility>

#include "mc.h"
#include "mc_direct.h"
#include "mc_internal.h"

namespace mc {
namespace {

constexpr int kDRhoChunk = 16;

// rho1 slot J of the chunk at J0: phase 0 target, 1 gather, 2 accumulate.
template <int MT, int J>
__device__ __forceinline__ int32_t drho1_target(const DirectRow<MT> &row, const int (&n)[MT])
{
    constexpr int k = J / MT, l = J % MT;
    if constexpr (k == l) return -1;
    else return n[k] >= 1 ? (int32_t)row.template target<k, -1, l, -1>() : -1;
}

template <int MT, bool BIGC, int J0, int... Is>
__device__ __forceinline__ void drho1_tile(std::integer_sequence<int, Is...>,
                                           const DirectRow<MT> &row, const int (&n)[MT],
                                           double2 cg, const Gather<BIGC> &ldc, const double *sq,
                                           double (&ar)[sizeof...(Is)], double (&ai)[sizeof...(Is)])
{
    constexpr int CH = sizeof...(Is);
    int32_t t[CH];
    double2 c[CH];
    ((t[Is] = drho1_target<MT, J0 + Is>(row, n)), ...);
    ((c[Is] = ldc(t[Is])), ...);
    (
        [&] {
            constexpr int k = (J0 + Is) / MT, l = (J0 + Is) % MT;
            if constexpr (k == l) {
                ar[Is] = fma(cg.x * cg.x + cg.y * cg.y, (double)n[k], ar[Is]);
            } else {
                const double f = sq[n[k]] * sq[n[l] + 1];
                ar[Is] = fma(cg.x * c[Is].x + cg.y * c[Is].y, f, ar[Is]);
                ai[Is] = fma(cg.x * c[Is].y - cg.y * c[Is].x, f, ai[Is]);
            }
        }(),
        ...);
}

template <int MT, bool BIGC, int J0>
__device__ __forceinline__ void drho1_chunk(int N, int nbits, int64_t D, int64_t tiles,
                                            int nwaves, int wave, const Gather<BIGC> &ldc,
                                            const double *sq, double2 *__restrict__ part)
{
    constexpr int NS = MT * MT;
    constexpr int CH = NS - J0 < kDRhoChunk ? NS - J0 : kDRhoChunk;
    const int lane = threadIdx.x & 63;
    double ar[CH], ai[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) ar[i] = ai[i] = 0.0;
    for (int64_t tile = wave; tile < tiles; tile += nwaves) {
        const int64_t g = tile * kTile + lane;
        const bool live = g < D;
        int n[MT];
        DirectRow<MT> row;
        row.init(live ? g : D - 1, D, N, nbits, n);
        const double2 cg = ldc(live ? (int32_t)g : -1);   // 0 on dead lanes
        drho1_tile<MT, BIGC, J0>(std::make_integer_sequence<int, CH>{}, row, n, cg, ldc, sq, ar,
                                 ai);
    }
#pragma unroll
    for (int i = 0; i < CH; ++i) {
        const double vr = wave_sum(ar[i]), vi = wave_sum(ai[i]);
        if (lane == 0) part[(int64_t)wave * NS + J0 + i] = make_double2(vr, vi);
    }
}

template <int MT, bool BIGC, int... Cs>
__device__ __forceinline__ void drho1_all(std::integer_sequence<int, Cs...>, int N, int nbits,
                                          int64_t D, int64_t tiles, int nwaves, int wave,
                                          const Gather<BIGC> &ldc, const double *sq,
                                          double2 *__restrict__ part)
{
    (drho1_chunk<MT, BIGC, Cs * kDRhoChunk>(N, nbits, D, tiles, nwaves, wave, ldc, sq, part), ...);
}

template <int MT, bool BIGC>
__global__ __launch_bounds__(256) void k_drho1(int N, int nbits, int64_t D, int64_t tiles,
                                                int nwaves, const double2 *__restrict__ C,
                                                double2 *__restrict__ part)
{
    extern __shared__ double sq[];
    fill_sqrt_table(sq, N + 3);
    const int wave = blockIdx.x * 4 + wave_in_block();
    if (wave >= nwaves) return;
    const Gather<BIGC> ldc(C, D);
    constexpr int NCH = (MT * MT + kDRhoChunk - 1) / kDRhoChunk;
    drho1_all<MT, BIGC>(std::make_integer_sequence<int, NCH>{}, N, nbits, D, tiles, nwaves, wave,
                        ldc, sq, part);
}

// rho2: removal pair P = (K, S), creation pair Q = (q, l), both unordered.
template <int MT, int P, int Q>
__device__ __forceinline__ int32_t drho2_target(const DirectRow<MT> &row, bool valid)
{
    constexpr int K = pair_k(MT, P), S = pair_s(MT, P), q = pair_k(MT, Q), l = pair_s(MT, Q);
    return valid ? (int32_t)row.template target<K, S, q, l>() : -1;
}

template <int MT, int P, int J0, int... Is>
__device__ __forceinline__ void drho2_tile(std::integer_sequence<int, Is...>,
                                           const DirectRow<MT> &row, const int (&n)[MT],
                                           bool valid, double xr, double xi,
                                           const Gather<false> &ldc, const double *sq,
                                           double (&ar)[sizeof...(Is)], double (&ai)[sizeof...(Is)])
{
    constexpr int CH = sizeof...(Is);
    constexpr int K = pair_k(MT, P), S = pair_s(MT, P);
    int32_t t[CH];
    double2 c[CH];
    ((t[Is] = drho2_target<MT, P, J0 + Is>(row, valid)), ...);
    ((c[Is] = ldc(t[Is])), ...);
    (
        [&] {
            constexpr int q = pair_k(MT, J0 + Is), l = pair_s(MT, J0 + Is);
            // creation amplitudes on m = n - e_K - e_S (rows with A = 0 may go below 0)
            const int mq = max(n[q] - (q == K) - (q == S), 0);
            const int ml = max(n[l] - (l == K) - (l == S), 0);
            const double B = q == l ? sq[mq + 1] * sq[mq + 2] : sq[mq + 1] * sq[ml + 1];
            const double pr = xr * c[Is].x - xi * c[Is].y, pi = xr * c[Is].y + xi * c[Is].x;
            ar[Is] = fma(pr, B, ar[Is]);
            ai[Is] = fma(pi, B, ai[Is]);
        }(),
        ...);
}

template <int MT, int P, int J0>
__device__ __forceinline__ void drho2_chunk(int N, int nbits, int64_t D, int64_t tiles,
                                            int nwaves, int wave, const Gather<false> &ldc,
                                            const double *sq, double2 *__restrict__ part)
{
    constexpr int NP = MT * (MT + 1) / 2, E = NP * NP;
    constexpr int K = pair_k(MT, P), S = pair_s(MT, P);
    constexpr int CH = NP - J0 < kDRhoChunk ? NP - J0 : kDRhoChunk;
    const int lane = threadIdx.x & 63;
    double ar[CH], ai[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) ar[i] = ai[i] = 0.0;
    for (int64_t tile = wave; tile < tiles; tile += nwaves) {
        const int64_t g = tile * kTile + lane;
        const bool live = g < D;
        int n[MT];
        DirectRow<MT> row;
        row.init(live ? g : D - 1, D, N, nbits, n);
        const bool valid = live && (K == S ? n[K] >= 2 : (n[K] >= 1 && n[S] >= 1));
        if (!__ballot(valid)) continue;   // no row of the tile can lose (K, S)
        const double2 cg = ldc(live ? (int32_t)g : -1);
        const double A = valid ? sq[n[K]] * (K == S ? sq[n[K] - 1] : sq[n[S]]) : 0.0;
        drho2_tile<MT, P, J0>(std::make_integer_sequence<int, CH>{}, row, n, valid, cg.x * A,
                              -cg.y * A, ldc, sq, ar, ai);
    }
#pragma unroll
    for (int i = 0; i < CH; ++i) {
        const double vr = wave_sum(ar[i]), vi = wave_sum(ai[i]);
        if (lane == 0) part[(int64_t)wave * E + P * NP + J0 + i] = make_double2(vr, vi);
    }
}

template <int MT, int P, int... Cs>
__device__ __forceinline__ void drho2_pair(std::integer_sequence<int, Cs...>, int N, int nbits,
                                           int64_t D, int64_t tiles, int nwaves, int wave,
                                           const Gather<false> &ldc, const double *sq,
                                           double2 *__restrict__ part)
{
    (drho2_chunk<MT, P, Cs * kDRhoChunk>(N, nbits, D, tiles, nwaves, wave, ldc, sq, part), ...);
}

template <int MT, int... Ps>
__device__ __forceinline__ void drho2_all(std::integer_sequence<int, Ps...>, int N, int nbits,
                                          int64_t D, int64_t tiles, int nwaves, int wave,
                                          const Gather<false> &ldc, const double *sq,
                                          double2 *__restrict__ part)
{
    constexpr int NCH = (MT * (MT + 1) / 2 + kDRhoChunk - 1) / kDRhoChunk;
    (drho2_pair<MT, Ps>(std::make_integer_sequence<int, NCH>{}, N, nbits, D, tiles, nwaves, wave,
                        ldc, sq, part),
     ...);
}

template <int MT>
__global__ __launch_bounds__(256) void k_drho2(int N, int nbits, int64_t D, int64_t tiles,
                                                int nwaves, const double2 *__restrict__ C,
                                                double2 *__restrict__ part)
{
    extern __shared__ double sq[];
    fill_sqrt_table(sq, N + 3);
    const int wave = blockIdx.x * 4 + wave_in_block();
    if (wave >= nwaves) return;
    const Gather<false> ldc(C, D);
    drho2_all<MT>(std::make_integer_sequence<int, MT * (MT + 1) / 2>{}, N, nbits, D, tiles, nwaves,
                  wave, ldc, sq, part);
}

// out[e] = sum over waves of part[w][e], in increasing w
__global__ void k_drho1_finalize(int E, int nwaves, const double2 *__restrict__ part,
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

// rho2[k][s][q][l] from the partials of the unordered pairs {k, s}, {q, l}
__global__ void k_drho2_finalize(int M, int nwaves, const double2 *__restrict__ part,
                                 double2 *__restrict__ out)
{
    const int total = M * M * M * M;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int l = idx % M, q = (idx / M) % M, s = (idx / (M * M)) % M, k = idx / (M * M * M);
    auto pair_of = [M](int x, int y) {
        const int a = x < y ? x : y, b = x < y ? y : x;
        return a * M - a * (a - 1) / 2 + (b - a);
    };
    const int NP = M * (M + 1) / 2;
    const int E = NP * NP;
    const int e = pair_of(k, s) * NP + pair_of(q, l);
    double sr = 0.0, si = 0.0;
    for (int w = 0; w < nwaves; ++w) {
        const double2 v = part[(int64_t)w * E + e];
        sr += v.x;
        si += v.y;
    }
    out[idx] = make_double2(sr, si);
}

constexpr int kDRhoMaxWaves = 4096;

// Common checks; *D_out, *nw_out on success.  The wave count is bounded by
// the workspace the caller passed, so partials never leave it.
int drho_setup(int32_t N, int32_t M, const double *C_d, const double *out_d, const void *ws_d,
               size_t ws_bytes, int op, int64_t *D_out, int *nw_out)
{
    int st = check_nm(N, M);
    if (st) return st;
    if (M > 8) return MC_EINVAL;
    const int64_t D = dim_checked(N, M);
    if (D < 0 || D >= ((int64_t)1 << 31)) return MC_ERANGE;
    if (!C_d || !out_d || !ws_d) return MC_EINVAL;
    if ((size_t)(N + 3) * 8 > 65536) return MC_EINVAL;
    size_t need = 0;
    mc_workspace_size(N, M, op, &need);
    if (ws_bytes < need) return MC_ENOMEM;
    const int64_t E = op == MC_OP_RHO1 ? (int64_t)M * M : (int64_t)npairs(M) * npairs(M);
    const int64_t tiles = (D + kTile - 1) / kTile;
    int64_t nw = tiles < kDRhoMaxWaves ? tiles : kDRhoMaxWaves;
    const int64_t fit = (int64_t)(ws_bytes / (size_t)(E * 16));
    if (nw > fit) nw = fit;
    if (nw < 1) return MC_ENOMEM;
    *D_out = D;
    *nw_out = (int)nw;
    return MC_OK;
}

}  // namespace
}  // namespace mc

using namespace mc;

extern "C" {

int mc_rho1_direct(int32_t N, int32_t M, const double *C_d, double *rho1_d, void *ws_d,
                   size_t ws_bytes, mc_stream stream)
{
    int64_t D = 0;
    int nw = 0;
    const int st = drho_setup(N, M, C_d, rho1_d, ws_d, ws_bytes, MC_OP_RHO1, &D, &nw);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    const int64_t tiles = (D + kTile - 1) / kTile;
    const int nbits = bit_width(N);
    const bool big = D * 16 > (int64_t)0xFFFFFFFFu;
    double2 *part = (double2 *)ws_d;
    const size_t sqb = (size_t)(N + 3) * 8;
    MC_DISPATCH_M(M, if constexpr (MT > 0 && MT <= 8) {
        if (big)
            hipLaunchKernelGGL((k_drho1<MT, true>), dim3((nw + 3) / 4), dim3(256), sqb, s, N, nbits,
                               D, tiles, nw, (const double2 *)C_d, part);
        else
            hipLaunchKernelGGL((k_drho1<MT, false>), dim3((nw + 3) / 4), dim3(256), sqb, s, N,
                               nbits, D, tiles, nw, (const double2 *)C_d, part);
    });
    hipLaunchKernelGGL(k_drho1_finalize, dim3((M * M + 255) / 256), dim3(256), 0, s, M * M, nw,
                       part, (double2 *)rho1_d);
    return launch_status();
}

int mc_rho2_direct(int32_t N, int32_t M, const double *C_d, double *rho2_d, void *ws_d,
                   size_t ws_bytes, mc_stream stream)
{
    int64_t D = 0;
    int nw = 0;
    const int st = drho_setup(N, M, C_d, rho2_d, ws_d, ws_bytes, MC_OP_RHO2, &D, &nw);
    if (st) return st;
    if (D * 16 > (int64_t)0xFFFFFFFFu) return MC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int64_t tiles = (D + kTile - 1) / kTile;
    const int nbits = bit_width(N);
    double2 *part = (double2 *)ws_d;
    const size_t sqb = (size_t)(N + 3) * 8;
    MC_DISPATCH_M(M, if constexpr (MT > 0 && MT <= 8) {
        hipLaunchKernelGGL((k_drho2<MT>), dim3((nw + 3) / 4), dim3(256), sqb, s, N, nbits, D, tiles,
                           nw, (const double2 *)C_d, part);
    });
    const int total = M * M * M * M;
    hipLaunchKernelGGL(k_drho2_finalize, dim3((total + 255) / 256), dim3(256), 0, s, M, nw, part,
                       (double2 *)rho2_d);
    return launch_status();
}

}  // extern "C"
