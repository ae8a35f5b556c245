// Hashing table and jump maps (paper Secs. III and IV) built on the device.
//
// Layout (see mc.h): every table is stored in 64-row tiles, one wavefront lane
// per row, so that the apply kernel reads 64 consecutive entries per load.
// Build order:
//   k_binom        B(x, m) = C(x+m, m) for x <= N+2, m <= M
//   k_build_index  per tile: unhash each row -> occupations, single-jump map,
//                  removal-pair mask (ballot over the tile), double-jump block
//                  length
//   k_scan_offsets exclusive prefix sum of block lengths -> t2_off
//   k_build_t2     per tile: for each pair in the mask, M*M*64 entries
#include <string.h>

#include "mc_internal.h"

namespace mc {

__global__ void k_binom(int N, int M, int64_t *__restrict__ binom)
{
    // one thread per column m: Pascal's rule B(x, m) = B(x-1, m) + B(x, m-1)
    // computed down the column after column m-1 is complete.  Tiny table,
    // one block; columns are produced in order with a barrier in between.
    const int M1 = M + 1;
    const int X = N + 3;
    for (int m = 0; m <= M; ++m) {
        for (int x = threadIdx.x; x < X; x += blockDim.x) {
            if (m == 0) binom[x * M1] = 1;
        }
        __syncthreads();
        if (m > 0 && threadIdx.x == 0) {
            int64_t acc = 0;
            for (int x = 0; x < X; ++x) {
                // B(x, m) = sum_{j<=x} B(j, m-1)  (hockey stick), saturating
                const int64_t v = binom[x * M1 + m - 1];
                acc = (acc > INT64_MAX - v) ? INT64_MAX : acc + v;
                binom[x * M1 + m] = acc;
            }
        }
        __syncthreads();
    }
}

template <int MT, typename OccT>
__global__ __launch_bounds__(256) void k_build_index(int N, int Mrt, int form, int64_t D,
                                                      int64_t tiles,
                                                      const int64_t *__restrict__ binom,
                                                      OccT *__restrict__ occ,
                                                      int32_t *__restrict__ t1,
                                                      uint64_t *__restrict__ pmask,
                                                      int64_t *__restrict__ t2_len)
{
    constexpr int MA = MT > 0 ? MT : MC_MAX_M;
    const int M = MT > 0 ? MT : Mrt;
    const int lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave_in_block();
    if (tile >= tiles) return;   // uniform per wavefront
    const int64_t g = tile * kTile + lane;
    int n[MA];
#pragma unroll (kUnroll<MT>)
    for (int m = 0; m < MA; ++m) n[m] = 0;
    if (g < D) dev_unhash<MT>(g, N, M, binom, n);

    for (int m = 0; m < M; ++m) occ[(tile * M + m) * kTile + lane] = (OccT)n[m];

    int w[MA];
    for (int k = 0; k < M; ++k) {
        for (int l = 0; l < M; ++l) {
            int32_t v = -1;
            if (n[k] >= 1) {
                if (k == l) {
                    v = (int32_t)g;
                } else {
#pragma unroll (kUnroll<MT>)
                    for (int m = 0; m < MA; ++m) w[m] = n[m];
                    w[k] -= 1;
                    w[l] += 1;
                    v = (int32_t)dev_hash<MT>(w, M, binom);
                }
            }
            t1[((tile * M + k) * M + l) * kTile + lane] = v;
        }
    }

    const int W = (M * (M + 1) / 2 + 63) / 64;
    uint64_t word = 0;
    int64_t slots = 0;
    int p = 0;
    for (int k = 0; k < M; ++k) {
        for (int s = k; s < M; ++s, ++p) {
            const unsigned long long b = __ballot(pair_valid(n, k, s));
            if (b) {
                word |= (uint64_t)1 << (p & 63);
                slots += form == MC_FORM_REDUCED ? reduced_slots(M, k, s) : M * M;
            }
            if ((p & 63) == 63) {
                if (lane == 0) pmask[tile * W + (p >> 6)] = word;
                word = 0;
            }
        }
    }
    if ((p & 63) != 0 && lane == 0) pmask[tile * W + (p >> 6)] = word;
    if (lane == 0) t2_len[tile] = slots * kTile;
}

// Exclusive scan of tiles+1 int64 values in place (the last input is
// ignored and receives the total).  One block; each thread scans a
// contiguous run of ITEMS values per round.
__global__ __launch_bounds__(1024) void k_scan_offsets(int64_t *__restrict__ a, int64_t n)
{
    constexpr int ITEMS = 8;
    __shared__ int64_t sums[1024];
    __shared__ int64_t carry_s;
    const int tid = threadIdx.x;
    if (tid == 0) carry_s = 0;
    __syncthreads();
    const int64_t chunk = (int64_t)blockDim.x * ITEMS;
    for (int64_t base = 0; base < n; base += chunk) {
        int64_t v[ITEMS];
        int64_t local = 0;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int64_t idx = base + (int64_t)tid * ITEMS + i;
            v[i] = idx < n - 1 ? a[idx] : 0;
            local += v[i];
        }
        sums[tid] = local;
        __syncthreads();
        // Hillis-Steele inclusive scan of the per-thread sums
        for (int o = 1; o < (int)blockDim.x; o <<= 1) {
            const int64_t add = tid >= o ? sums[tid - o] : 0;
            __syncthreads();
            sums[tid] += add;
            __syncthreads();
        }
        int64_t run = carry_s + sums[tid] - local;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int64_t idx = base + (int64_t)tid * ITEMS + i;
            if (idx < n) a[idx] = run;
            run += v[i];
        }
        __syncthreads();
        if (tid == (int)blockDim.x - 1) carry_s = run;
        __syncthreads();
    }
}

template <int MT, typename OccT>
__global__ __launch_bounds__(256) void k_build_t2(int N, int Mrt, int64_t tiles,
                                                   const int64_t *__restrict__ binom,
                                                   const OccT *__restrict__ occ,
                                                   const uint64_t *__restrict__ pmask,
                                                   const int64_t *__restrict__ t2_off,
                                                   int64_t cap, int32_t *__restrict__ t2)
{
    constexpr int MA = MT > 0 ? MT : MC_MAX_M;
    const int M = MT > 0 ? MT : Mrt;
    const int lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave_in_block();
    if (tile >= tiles) return;
    int n[MA], w[MA];
#pragma unroll (kUnroll<MT>)
    for (int m = 0; m < MA; ++m) n[m] = 0;
    for (int m = 0; m < M; ++m) n[m] = (int)occ[(tile * M + m) * kTile + lane];
    const int W = (M * (M + 1) / 2 + 63) / 64;
    // the block must hold exactly (pairs in the mask) * M*M*64 entries inside
    // the table; otherwise write nothing (the offsets are then corrupt)
    int64_t pairs = 0;
    for (int j = 0; j < W; ++j) pairs += __popcll(pmask[tile * W + j]);
    int64_t off0, off1;
    t2_block(t2_off, tile, cap, off0, off1);
    if (off1 - off0 != pairs * M * M * kTile) return;
    int32_t *dst = t2 + off0;
    int p = 0;
    int64_t rank = 0;
    for (int k = 0; k < M; ++k) {
        for (int s = k; s < M; ++s, ++p) {
            const uint64_t word = pmask[tile * W + (p >> 6)];
            if (!((word >> (p & 63)) & 1)) continue;
            const bool valid = pair_valid(n, k, s);
            int32_t *blk = dst + rank * M * M * kTile;
            for (int q = 0; q < M; ++q) {
                for (int l = 0; l < M; ++l) {
                    int32_t v = -1;
                    if (valid) {
#pragma unroll (kUnroll<MT>)
                        for (int m = 0; m < MA; ++m) w[m] = n[m];
                        w[k] -= 1;
                        w[s] -= 1;
                        w[q] += 1;
                        w[l] += 1;
                        v = (int32_t)dev_hash<MT>(w, M, binom);
                    }
                    blk[(q * M + l) * kTile + lane] = v;
                }
            }
            ++rank;
        }
    }
}

// Reduced double-jump map (true double jumps only), same tiling as k_build_t2
// with nd(k, s) slots per present pair.
template <int MT, typename OccT>
__global__ __launch_bounds__(256) void k_build_t2r(int N, int Mrt, int64_t tiles,
                                                    const int64_t *__restrict__ binom,
                                                    const OccT *__restrict__ occ,
                                                    const uint64_t *__restrict__ pmask,
                                                    const int64_t *__restrict__ t2_off,
                                                    int64_t cap, int32_t *__restrict__ t2)
{
    constexpr int MA = MT > 0 ? MT : MC_MAX_M;
    const int M = MT > 0 ? MT : Mrt;
    const int lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave_in_block();
    if (tile >= tiles) return;
    int n[MA], w[MA];
#pragma unroll (kUnroll<MT>)
    for (int m = 0; m < MA; ++m) n[m] = 0;
    for (int m = 0; m < M; ++m) n[m] = (int)occ[(tile * M + m) * kTile + lane];
    const int W = (M * (M + 1) / 2 + 63) / 64;
    // the tile's block must be exactly the sum of its present pairs' slots
    int64_t want = 0;
    {
        int p = 0;
        for (int k = 0; k < M; ++k)
            for (int s = k; s < M; ++s, ++p)
                if ((pmask[tile * W + (p >> 6)] >> (p & 63)) & 1) want += reduced_slots(M, k, s);
    }
    int64_t off0, off1;
    t2_block(t2_off, tile, cap, off0, off1);
    if (off1 - off0 != want * kTile) return;
    int32_t *dst = t2 + off0;
    int p = 0;
    for (int k = 0; k < M; ++k) {
        for (int s = k; s < M; ++s, ++p) {
            const uint64_t word = pmask[tile * W + (p >> 6)];
            if (!((word >> (p & 63)) & 1)) continue;
            const bool valid = pair_valid(n, k, s);
            int r = 0;
            for (int q = 0; q < M; ++q) {
                for (int l = q; l < M; ++l) {
                    if (q == k || q == s || l == k || l == s) continue;
                    int32_t v = -1;
                    if (valid) {
#pragma unroll (kUnroll<MT>)
                        for (int m = 0; m < MA; ++m) w[m] = n[m];
                        w[k] -= 1;
                        w[s] -= 1;
                        w[q] += 1;
                        w[l] += 1;
                        v = (int32_t)dev_hash<MT>(w, M, binom);
                    }
                    dst[r * kTile + lane] = v;
                    ++r;
                }
            }
            dst += (int64_t)r * kTile;
        }
    }
}

template <int MT>
__global__ void k_hash_batch(int N, int Mrt, const int64_t *__restrict__ binom,
                             const int32_t *__restrict__ occ, int64_t *__restrict__ idx,
                             int64_t count)
{
    constexpr int MA = MT > 0 ? MT : MC_MAX_M;
    const int M = MT > 0 ? MT : Mrt;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    int n[MA];
#pragma unroll (kUnroll<MT>)
    for (int m = 0; m < MA; ++m) n[m] = 0;
    int64_t sum = 0;
    bool ok = true;
    for (int m = 0; m < M; ++m) {
        n[m] = occ[i * M + m];
        ok = ok && n[m] >= 0 && n[m] <= N;
        sum += n[m];
    }
    idx[i] = (ok && sum == N) ? dev_hash<MT>(n, M, binom) : -1;
}

template <int MT>
__global__ void k_unhash_batch(int N, int Mrt, int64_t D, const int64_t *__restrict__ binom,
                               const int64_t *__restrict__ idx, int32_t *__restrict__ occ,
                               int64_t count)
{
    constexpr int MA = MT > 0 ? MT : MC_MAX_M;
    const int M = MT > 0 ? MT : Mrt;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t r = idx[i];
    int n[MA];
#pragma unroll (kUnroll<MT>)
    for (int m = 0; m < MA; ++m) n[m] = -1;
    if (r >= 0 && r < D) dev_unhash<MT>(r, N, M, binom, n);
    for (int m = 0; m < M; ++m) occ[i * M + m] = n[m];
}

template <typename OccT>
__global__ void k_t2_lookup(int M, int64_t D, const OccT *__restrict__ occ,
                            const uint64_t *__restrict__ pmask,
                            const int64_t *__restrict__ t2_off, int64_t cap,
                            const int32_t *__restrict__ t2, const int64_t *__restrict__ q5,
                            int32_t *__restrict__ out, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t row = q5[i * 5 + 0];
    int64_t k = q5[i * 5 + 1], s = q5[i * 5 + 2];
    const int64_t q = q5[i * 5 + 3], l = q5[i * 5 + 4];
    int32_t v = -1;
    if (row >= 0 && row < D && k >= 0 && k < M && s >= 0 && s < M && q >= 0 && q < M && l >= 0 &&
        l < M) {
        if (k > s) { const int64_t t = k; k = s; s = t; }
        const int64_t tile = row / kTile, lane = row % kTile;
        const int nk = occ[(tile * M + k) * kTile + lane];
        const int ns = occ[(tile * M + s) * kTile + lane];
        const bool valid = k == s ? nk >= 2 : (nk >= 1 && ns >= 1);
        if (valid) {
            const int W = (M * (M + 1) / 2 + 63) / 64;
            // pair index of (k, s) in lexicographic k <= s order
            const int64_t p = k * M - k * (k - 1) / 2 + (s - k);
            int64_t rank = 0;
            for (int64_t j = 0; j < p; ++j)
                rank += (pmask[tile * W + (j >> 6)] >> (j & 63)) & 1;
            int64_t off0, off1;
            t2_block(t2_off, tile, cap, off0, off1);
            const int64_t pos = off0 + ((rank * M + q) * M + l) * kTile + lane;
            v = pos < off1 ? t2[pos] : -1;
        }
    }
    out[i] = v;
}

}  // namespace mc

using namespace mc;

extern "C" {

int mc_build_jump_tables(int32_t N, int32_t M, mc_tables *t, mc_stream stream)
{
    int st = check_nm(N, M);
    if (st) return st;
    st = check_tables(N, M, t, false);
    if (st) return st;
    if (t->dim >= ((int64_t)1 << 31)) return MC_ERANGE;
    hipStream_t s = (hipStream_t)stream;
    const int64_t D = t->dim, tiles = t->tiles;
    hipLaunchKernelGGL(k_binom, dim3(1), dim3(256), 0, s, N, M, t->binom_d);
    const int64_t blocks = (tiles + 3) / 4;
    if (occ_width(N) == 1) {
        MC_DISPATCH_M(M, hipLaunchKernelGGL((k_build_index<MT, uint8_t>), dim3(blocks), dim3(256),
                                            0, s, N, M, t->form, D, tiles, t->binom_d,
                                            (uint8_t *)t->occ_d, t->t1_d, t->pmask_d,
                                            t->t2_off_d));
    } else {
        MC_DISPATCH_M(M, hipLaunchKernelGGL((k_build_index<MT, uint16_t>), dim3(blocks),
                                            dim3(256), 0, s, N, M, t->form, D, tiles, t->binom_d,
                                            (uint16_t *)t->occ_d, t->t1_d, t->pmask_d,
                                            t->t2_off_d));
    }
    hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(1024), 0, s, t->t2_off_d, tiles + 1);
    st = launch_status();
    if (st) return st;
    int64_t total = 0;
    st = set_hip_error(hipMemcpyAsync(&total, t->t2_off_d + tiles, sizeof(total),
                                      hipMemcpyDeviceToHost, s));
    if (st) return st;
    st = set_hip_error(hipStreamSynchronize(s));
    if (st) return st;
    t->t2_required = total;
    return MC_OK;
}

int mc_build_double_jumps(int32_t N, int32_t M, const mc_tables *t, mc_stream stream)
{
    int st = check_nm(N, M);
    if (st) return st;
    st = check_tables(N, M, t, true);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    const int64_t blocks = (t->tiles + 3) / 4;
    if (t->form == MC_FORM_REDUCED) {
        if (occ_width(N) == 1) {
            MC_DISPATCH_M(M, hipLaunchKernelGGL((k_build_t2r<MT, uint8_t>), dim3(blocks),
                                                dim3(256), 0, s, N, M, t->tiles, t->binom_d,
                                                (const uint8_t *)t->occ_d, t->pmask_d,
                                                t->t2_off_d, t->t2_entries, t->t2_d));
        } else {
            MC_DISPATCH_M(M, hipLaunchKernelGGL((k_build_t2r<MT, uint16_t>), dim3(blocks),
                                                dim3(256), 0, s, N, M, t->tiles, t->binom_d,
                                                (const uint16_t *)t->occ_d, t->pmask_d,
                                                t->t2_off_d, t->t2_entries, t->t2_d));
        }
        return launch_status();
    }
    if (occ_width(N) == 1) {
        MC_DISPATCH_M(M, hipLaunchKernelGGL((k_build_t2<MT, uint8_t>), dim3(blocks), dim3(256), 0,
                                            s, N, M, t->tiles, t->binom_d,
                                            (const uint8_t *)t->occ_d, t->pmask_d, t->t2_off_d,
                                            t->t2_entries, t->t2_d));
    } else {
        MC_DISPATCH_M(M, hipLaunchKernelGGL((k_build_t2<MT, uint16_t>), dim3(blocks), dim3(256),
                                            0, s, N, M, t->tiles, t->binom_d,
                                            (const uint16_t *)t->occ_d, t->pmask_d, t->t2_off_d,
                                            t->t2_entries, t->t2_d));
    }
    return launch_status();
}

int mc_hash_batch(int32_t N, int32_t M, const mc_tables *t, const int32_t *occ_d,
                  int64_t *index_d, int64_t count, mc_stream stream)
{
    int st = check_nm(N, M);
    if (st) return st;
    if (!t || t->N != N || t->M != M || !t->binom_d || count < 0) return MC_EINVAL;
    if (count == 0) return MC_OK;
    if (!occ_d || !index_d) return MC_EINVAL;
    const int64_t blocks = (count + 255) / 256;
    MC_DISPATCH_M(M, hipLaunchKernelGGL((k_hash_batch<MT>), dim3(blocks), dim3(256), 0,
                                        (hipStream_t)stream, N, M, t->binom_d, occ_d, index_d,
                                        count));
    return launch_status();
}

int mc_unhash_batch(int32_t N, int32_t M, const mc_tables *t, const int64_t *index_d,
                    int32_t *occ_d, int64_t count, mc_stream stream)
{
    int st = check_nm(N, M);
    if (st) return st;
    if (!t || t->N != N || t->M != M || !t->binom_d || count < 0) return MC_EINVAL;
    if (count == 0) return MC_OK;
    if (!occ_d || !index_d) return MC_EINVAL;
    const int64_t D = dim_checked(N, M);
    const int64_t blocks = (count + 255) / 256;
    MC_DISPATCH_M(M, hipLaunchKernelGGL((k_unhash_batch<MT>), dim3(blocks), dim3(256), 0,
                                        (hipStream_t)stream, N, M, D, t->binom_d, index_d, occ_d,
                                        count));
    return launch_status();
}

int mc_t2_lookup(int32_t N, int32_t M, const mc_tables *t, const int64_t *queries_d,
                 int32_t *out_d, int64_t count, mc_stream stream)
{
    int st = check_nm(N, M);
    if (st) return st;
    st = check_tables(N, M, t, true);
    if (st) return st;
    if (t->form != MC_FORM_PAPER || count < 0) return MC_EINVAL;
    if (count == 0) return MC_OK;
    if (!queries_d || !out_d) return MC_EINVAL;
    const int64_t blocks = (count + 255) / 256;
    if (occ_width(N) == 1)
        hipLaunchKernelGGL((k_t2_lookup<uint8_t>), dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                           M, t->dim, (const uint8_t *)t->occ_d, t->pmask_d, t->t2_off_d,
                           t->t2_entries, t->t2_d,
                           queries_d, out_d, count);
    else
        hipLaunchKernelGGL((k_t2_lookup<uint16_t>), dim3(blocks), dim3(256), 0,
                           (hipStream_t)stream, M, t->dim, (const uint16_t *)t->occ_d, t->pmask_d,
                           t->t2_off_d, t->t2_entries, t->t2_d, queries_d, out_d, count);
    return launch_status();
}

}  // extern "C"
