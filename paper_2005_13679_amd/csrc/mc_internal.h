// Internal helpers shared by the HIP translation units of libmc.
//
// Index arithmetic.  With S_m = n_0 + ... + n_m, the cost that Eq. (TotalCost)
// assigns to the particles of orbital m telescopes (hockey-stick identity) to
//     sum_{s = S_{m-1}+1}^{S_m} C(s+m-1, m-1) = C(S_m + m, m) - C(S_{m-1} + m, m),
// so the index of a configuration is
//     I(n) = sum_{m=1}^{M-1} [ B(S_m, m) - B(S_{m-1}, m) ],   B(x, m) = C(x+m, m),
// an O(M) evaluation instead of the O(N) particle loop of Algorithm 1.
// The inverse walks orbitals from M-1 down: with S particles left in
// orbitals 0..m and remaining index r < B(S, m), the configurations with
// n_m = S - x start at B(S, m) - B(x, m); n_m follows from the smallest x
// with B(x, m) >= B(S, m) - r, found by binary search (the result agrees
// with Algorithm 2's greedy descent, which moves one particle at a time).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mc.h"

namespace mc {

// Full unrolling of orbital loops for a compile-time orbital count; loops
// stay rolled for the run-time (MT = 0) variants.
template <int MT>
constexpr int kUnroll = MT > 0 ? 32 : 1;

constexpr int kTile = MC_TILE;   // rows per tile = lanes per wavefront
constexpr int kWave = 64;

int set_hip_error(hipError_t e);        // records e, returns MC_EHIP (or MC_OK)
int launch_status();                   // hipGetLastError -> status

inline int npairs(int M) { return M * (M + 1) / 2; }
inline int pair_words(int M) { return (npairs(M) + 63) / 64; }
inline int occ_width(int N) { return N <= 255 ? 1 : 2; }
// number of bits of N (N >= 0)
inline int bit_width(int N)
{
    int b = 0;
    while (b < 31 && (1 << b) <= N) ++b;
    return b;
}
// Slots of removal pair (k, s) in the reduced double-jump map: creation
// pairs q <= l with q, l outside {k, s}.
__host__ __device__ constexpr int reduced_slots(int M, int k, int s)
{
    return k == s ? M * (M - 1) / 2 : (M - 1) * (M - 2) / 2;
}
// Staged constants of the case-split apply (complex entries): DL[M],
// GI[M(M+1)/2], HS[M*M], GS[M*M*M], GD[reduced slots of all pairs].
__host__ __device__ constexpr int split_dl_offset(int) { return 0; }
__host__ __device__ constexpr int split_gi_offset(int M) { return M; }
__host__ __device__ constexpr int split_hs_offset(int M) { return M + M * (M + 1) / 2; }
__host__ __device__ constexpr int split_gs_offset(int M) { return split_hs_offset(M) + M * M; }
__host__ __device__ constexpr int split_gd_offset(int M) { return split_gs_offset(M) + M * M * M; }
__host__ __device__ constexpr int split_total(int M)
{
    return split_gd_offset(M) + M * reduced_slots(M, 0, 0) +
           (M * (M - 1) / 2) * (M >= 2 ? reduced_slots(M, 0, 1) : 0);
}
// Entries of one full row of the reduced map (every pair valid).
inline int64_t reduced_row_entries(int M)
{
    return (int64_t)M * reduced_slots(M, 0, 0) +
           (int64_t)(M * (M - 1) / 2) * (M >= 2 ? reduced_slots(M, 0, 1) : 0);
}

// Workspace bytes of the table-free density matrices over configurations of
// N - L particles (L = 1: rho1, L = 2: rho2); 0 if a dimension overflows.
size_t gram_workspace(int32_t N, int32_t M, int L);
// The same through the jump maps (rows of the N-particle space).
size_t gram_table_workspace(int32_t N, int32_t M, int L);
// rho1 through the single-jump map for M > 8 (run-time orbital count).
int rho1_generic(int32_t N, int32_t M, const mc_tables *t, const double *C_d, double *rho1_d,
                 void *ws_d, size_t ws_bytes, mc_stream stream);

// Validates (N, M) ranges; MC_OK or MC_EINVAL.
int check_nm(int32_t N, int32_t M);
// D = C(N+M-1, N) with overflow check; -1 on overflow.
int64_t dim_checked(int32_t N, int32_t M);
// Validates a table descriptor against (N, M).  need_t2: t2 must be built.
int check_tables(int32_t N, int32_t M, const mc_tables *t, bool need_t2);
// True if [a, a+na) and [b, b+nb) (bytes) overlap.
bool overlaps(const void *a, size_t na, const void *b, size_t nb);

// Raw buffer resource for gfx9: hardware range check on num_records bytes,
// out-of-range loads return zero instead of faulting.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             0x00020000);
}

__device__ __forceinline__ int32_t buf_ld_i32(__amdgpu_buffer_rsrc_t r, uint32_t byte_off,
                                              uint32_t soff)
{
    // nt: table entries are streamed once per apply
    return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, (int)soff, 2);
}

__device__ __forceinline__ double2 buf_ld_c128(__amdgpu_buffer_rsrc_t r, uint32_t byte_off)
{
    auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)byte_off, 0, 0);
    double2 d;
    __builtin_memcpy(&d, &v, sizeof(d));
    return d;
}

// B(x, m) = C(x+m, m), row-major [x][m] with row stride M+1.
__device__ __forceinline__ int64_t binom_at(const int64_t *__restrict__ binom, int M1, int x,
                                            int m)
{
    return binom[x * M1 + m];
}

// Closed-form index of an occupation vector (see file header).
template <int MT>
__device__ __forceinline__ int64_t dev_hash(const int *n, int M, const int64_t *__restrict__ binom)
{
    const int Mr = MT > 0 ? MT : M;
    const int M1 = Mr + 1;
    int64_t idx = 0;
    int S = n[0];
#pragma unroll (kUnroll<MT>)
    for (int m = 1; m < (MT > 0 ? MT : MC_MAX_M); ++m) {
        if (MT == 0 && m >= Mr) break;
        const int Sp = S;
        S += n[m];
        idx += binom_at(binom, M1, S, m) - binom_at(binom, M1, Sp, m);
    }
    return idx;
}

// Inverse of dev_hash by per-orbital binary search (see file header).
template <int MT>
__device__ __forceinline__ void dev_unhash(int64_t r, int N, int M,
                                           const int64_t *__restrict__ binom, int *n)
{
    const int Mr = MT > 0 ? MT : M;
    const int M1 = Mr + 1;
    int S = N;
#pragma unroll (kUnroll<MT>)
    for (int m = (MT > 0 ? MT : MC_MAX_M) - 1; m >= 1; --m) {
        if (MT == 0 && m >= Mr) continue;
        const int64_t top = binom_at(binom, M1, S, m);
        const int64_t need = top - r;
        int lo = 0, hi = S;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (binom_at(binom, M1, mid, m) >= need) hi = mid;
            else lo = mid + 1;
        }
        n[m] = S - lo;
        r -= top - binom_at(binom, M1, lo, m);
        S = lo;
    }
    n[0] = S;
}

__device__ __forceinline__ bool pair_valid(const int *n, int k, int s)
{
    return k == s ? n[k] >= 2 : (n[k] >= 1 && n[s] >= 1);
}

// Wave-wide sum (all lanes receive the total).  Fixed butterfly order, so the
// result is deterministic.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// [off0, off1) of a tile's double-jump block, clamped to the table capacity
// so that corrupted offsets can never address memory outside the table.
__device__ __forceinline__ void t2_block(const int64_t *__restrict__ t2_off, int64_t tile,
                                         int64_t cap, int64_t &off0, int64_t &off1)
{
    off1 = t2_off[tile + 1];
    off0 = t2_off[tile];
    off1 = off1 < cap ? off1 : cap;
    off1 = off1 > 0 ? off1 : 0;
    off0 = off0 < off1 ? off0 : off1;
    off0 = off0 > 0 ? off0 : 0;
}

// Index of the calling wavefront within its block, as a wave-uniform (SGPR)
// value: the compiler cannot prove threadIdx.x >> 6 uniform by itself, and
// anything derived from a divergent value (tile, offsets, buffer resources)
// would force per-lane waterfall loops around every buffer load.
__device__ __forceinline__ int wave_in_block()
{
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// Maps a hardware block index to a logical one.  The 8 XCDs receive blocks
// round-robin.  With MC_XCD_REMAP = 1 each XCD works on one contiguous range
// of blocks; with MC_XCD_CHUNK = K > 1 (the default, remap off) each XCD takes
// contiguous chunks of K blocks, the chunks interleaved over the XCDs (blocks
// past the last whole group of 8K map to themselves).  Neighbouring tiles
// gather from overlapping coefficient windows, so chunks let one XCD's L2
// serve them, while interleaved chunks keep all XCDs in one region of the
// index space, whose windows the memory-side cache then shares.  Measured at
// N=200, M=5 against the identity (K = 1) and the full remap: K = 512 is
// 3 % (reduced map), 1.5 % (paper map), 6 % (no table) and 15 % (chained)
// faster than the identity; the full remap is 2-8 % slower than it.
#ifndef MC_XCD_REMAP
#define MC_XCD_REMAP 0
#endif
#ifndef MC_XCD_CHUNK
#define MC_XCD_CHUNK 512
#endif
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb)
{
    if (!MC_XCD_REMAP) {
        if (MC_XCD_CHUNK <= 1) return b;
        const int64_t full = nb / (8 * MC_XCD_CHUNK) * (8 * MC_XCD_CHUNK);
        if (b >= full) return b;
        const int64_t x = b & 7, i = b >> 3;
        return ((i / MC_XCD_CHUNK) * 8 + x) * MC_XCD_CHUNK + i % MC_XCD_CHUNK;
    }
    const int64_t xcd = b & 7, local = b >> 3;
    const int64_t per = nb >> 3, rem = nb & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
}

// The same with the mapping chosen per kernel: XCD-contiguous ranges (REMAP)
// or the build default.
template <bool REMAP>
__device__ __forceinline__ int64_t xcd_block_as(int64_t b, int64_t nb)
{
    if constexpr (!REMAP) return xcd_block(b, nb);
    const int64_t xcd = b & 7, local = b >> 3;
    const int64_t per = nb >> 3, rem = nb & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
}

}  // namespace mc

// Dispatch a templated kernel launch on a compile-time orbital count for
// M <= 8, with MT = 0 (run-time M) above that.
#define MC_DISPATCH_M(Mval, BODY)                          \
    switch (Mval) {                                        \
    case 1: { constexpr int MT = 1; BODY; } break;         \
    case 2: { constexpr int MT = 2; BODY; } break;         \
    case 3: { constexpr int MT = 3; BODY; } break;         \
    case 4: { constexpr int MT = 4; BODY; } break;         \
    case 5: { constexpr int MT = 5; BODY; } break;         \
    case 6: { constexpr int MT = 6; BODY; } break;         \
    case 7: { constexpr int MT = 7; BODY; } break;         \
    case 8: { constexpr int MT = 8; BODY; } break;         \
    default: { constexpr int MT = 0; BODY; } break;        \
    }
