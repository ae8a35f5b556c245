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
#include <mutex>
#include <utility>

#include "mc_apply.h"
#include "mc_split.h"
#include "mc_sparse.h"
#include "mc_direct.h"
#include "mc_gram.h"
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

// Staged constants of the case-split apply (layout in mc_split.h).
__global__ void k_prep_split(int M, int adjoint, const double2 *__restrict__ g,
                             const double2 *__restrict__ h, double2 *__restrict__ cf)
{
    stage_split_constants(M, adjoint, g, h, cf, blockIdx.x * blockDim.x + threadIdx.x,
                          gridDim.x * blockDim.x);
}

// H.C in the case-split form walking only the nonzero constants (lists
// built by k_sparse_lists); reduced tables, MAP as in k_apply_split.
template <int MT, typename OccT, bool BIGC, bool MAP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MC_APPLY_WAVES)))
void k_apply_sparse(int N, int64_t D, int64_t tiles, int64_t nblocks, int64_t cap,
                    const OccT *__restrict__ occ, const int32_t *__restrict__ t1,
                    const uint64_t *__restrict__ pmask, const int64_t *__restrict__ t2_off,
                    const int32_t *__restrict__ t2r, const double2 *__restrict__ cf,
                    const int32_t *__restrict__ sl, const double2 *__restrict__ C,
                    double2 *__restrict__ HC)
{
    extern __shared__ double sq[];
    fill_sqrt_table(sq, N + 3);
    const int64_t tile = xcd_block(blockIdx.x, nblocks) * 4 + wave_in_block();
    if (tile >= tiles) return;
    apply_tile_sparse<MT, OccT, BIGC, MAP>(tile, D, cap, sq, occ, t1, pmask, t2_off, t2r, cf, sl,
                                           C, HC);
}

// H.C in the case-split form (reduced tables); MAP: reduced double-jump map
// present, else chained single jumps.
template <int MT, typename OccT, bool BIGC, bool MAP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MC_APPLY_WAVES)))
void k_apply_split(int N, int64_t D, int64_t tiles, int64_t nblocks, int64_t cap,
                   const OccT *__restrict__ occ, const int32_t *__restrict__ t1,
                   const uint64_t *__restrict__ pmask, const int64_t *__restrict__ t2_off,
                   const int32_t *__restrict__ t2r, const double2 *__restrict__ cf,
                   const double2 *__restrict__ C, double2 *__restrict__ HC)
{
    extern __shared__ double sq[];
    if constexpr (kLdsRoots<MT>) fill_sqrt_table(sq, N + 3);
    const int64_t tile = xcd_block(blockIdx.x, nblocks) * 4 + wave_in_block();
    if (tile >= tiles) return;
    apply_tile_split<MT, OccT, BIGC, MAP>(tile, D, cap, sq, occ, t1, pmask, t2_off, t2r, cf, C, HC);
}

// H.C with no table (occupations and targets in closed form, mc_direct.h).
template <int MT, bool BIGC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MC_APPLY_WAVES)))
void k_apply_direct(int N, int nbits, int64_t D, int64_t tiles, int64_t nblocks,
                    const double2 *__restrict__ cf, const double2 *__restrict__ C,
                    double2 *__restrict__ HC)
{
    extern __shared__ double sq[];
    if constexpr (kLdsRoots<MT>) fill_sqrt_table(sq, N + 3);
    const int64_t tile = xcd_block_as<kDirectRemap<MT>>(blockIdx.x, nblocks) * 4 + wave_in_block();
    if (tile >= tiles) return;
    apply_tile_direct<MT, BIGC>(tile, N, nbits, D, sq, cf, C, HC);
}

template <int MT, typename OccT, bool BIGC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MC_APPLY_WAVES)))
void k_apply(int N, int64_t D, int64_t tiles, int64_t nblocks, int64_t cap,
             const OccT *__restrict__ occ, const int32_t *__restrict__ t1,
             const uint64_t *__restrict__ pmask, const int64_t *__restrict__ t2_off,
             const int32_t *__restrict__ t2, const double2 *__restrict__ h,
             const double2 *__restrict__ gp, const double2 *__restrict__ C,
             double2 *__restrict__ HC)
{
    extern __shared__ double sq[];
    if constexpr (kLdsRoots<MT>) fill_sqrt_table(sq, N + 3);
    const int64_t tile = xcd_block(blockIdx.x, nblocks) * 4 + wave_in_block();
    if (tile >= tiles) return;
    apply_tile_paper<MT, OccT, BIGC>(tile, D, cap, sq, occ, t1, pmask, t2_off, t2, h, gp, C, HC);
}

template <int MT, typename OccT, bool BIGC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MC_APPLY_WAVES)))
void k_apply_chained(int N, int64_t D, int64_t tiles, int64_t nblocks,
                     const OccT *__restrict__ occ, const int32_t *__restrict__ t1,
                     const double2 *__restrict__ h, const double2 *__restrict__ gp,
                     const double2 *__restrict__ C, double2 *__restrict__ HC)
{
    extern __shared__ double sq[];
    if constexpr (kLdsRoots<MT>) fill_sqrt_table(sq, N + 3);
    const int64_t tile = xcd_block(blockIdx.x, nblocks) * 4 + wave_in_block();
    if (tile >= tiles) return;
    apply_tile_chained<MT, OccT, BIGC>(tile, D, sq, occ, t1, h, gp, C, HC);
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
// rho1 for M > 8 (the Gram kernels of mc_gram.h cover M <= 8).  Wave w
// accumulates tiles w, w + nwaves, ... in a fixed order; each per-slot value
// is summed over the 64 rows of the tile with a butterfly (all lanes receive
// the total) and lane (e mod 64) keeps element e.  Partials per wave go to
// the workspace ([element][wave]) and are summed over waves by a fixed tree:
// results are bitwise reproducible.
// ---------------------------------------------------------------------------
constexpr int kRhoWaves = 4096;

inline int rho_waves(int64_t tiles) { return (int)(tiles < kRhoWaves ? tiles : kRhoWaves); }

template <int MT, typename OccT, bool BIGC>
__global__ __launch_bounds__(256) void k_rho1_generic(int Mrt, int64_t D, int64_t tiles, int nwaves,
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
        double s0[MA], sp1[MA];
#pragma unroll (kUnroll<MT>)
        for (int m = 0; m < MA; ++m) {
            if (MT == 0 && m >= M) break;
            n[m] = (int)occ[(tile * M + m) * kTile + lane];
            s0[m] = sqrt((double)n[m]);
            sp1[m] = sqrt((double)n[m] + 1.0);
        }
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
                    const double f = s0[k] * sp1[l];
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
        if (e < E) part[(int64_t)e * nwaves + wave] = make_double2(accr[j], acci[j]);
    }
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

// out[i] = sum_k V[k][i] c[k]  (the Krylov combination of a propagation step)
__global__ __launch_bounds__(256) void k_zgemv_n(int K, int64_t n, const double2 *__restrict__ V,
                                                  int64_t ldv, const double2 *__restrict__ c,
                                                  double2 *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double sr = 0.0, si = 0.0;
        for (int k = 0; k < K; ++k) {
            const double2 a = V[(int64_t)k * ldv + i], b = c[k];
            sr += a.x * b.x - a.y * b.y;
            si += a.x * b.y + a.y * b.x;
        }
        out[i] = make_double2(sr, si);
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

// flag[0] = 1 if h_kl == conj(h_lk) and g_ksql == conj(g_lqsk) for every
// index (exact comparisons; then H^dagger = H elementwise), else 0.
__global__ __launch_bounds__(256) void k_is_hermitian(int M, const double2 *__restrict__ h,
                                                      const double2 *__restrict__ g,
                                                      int32_t *__restrict__ flag)
{
    __shared__ int ok;
    if (threadIdx.x == 0) ok = 1;
    __syncthreads();
    int mine = 1;
    const int M2 = M * M;
    for (int e = threadIdx.x; e < M2; e += blockDim.x) {
        const int k = e / M, l = e % M;
        const double2 a = h[e], b = h[l * M + k];
        if (!(a.x == b.x && a.y == -b.y)) mine = 0;
    }
    const int M4 = M2 * M2;
    for (int e = threadIdx.x; e < M4; e += blockDim.x) {
        const int l = e % M, q = (e / M) % M, s = (e / M2) % M, k = e / (M2 * M);
        const double2 a = g[e], b = g[((l * M + q) * M + s) * M + k];
        if (!(a.x == b.x && a.y == -b.y)) mine = 0;
    }
    if (!mine) atomicAnd(&ok, 0);
    __syncthreads();
    if (threadIdx.x == 0) flag[0] = ok;
}

int rho1_generic(int32_t N, int32_t M, const mc_tables *t, const double *C_d, double *rho1_d,
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
    if (occ_width(N) == 1) {
        if (big)
            hipLaunchKernelGGL((k_rho1_generic<0, uint8_t, true>), dim3((nw + 3) / 4), dim3(256),
                               0, s, M, D, t->tiles, nw, (const uint8_t *)t->occ_d, t->t1_d,
                               (const double2 *)C_d, part);
        else
            hipLaunchKernelGGL((k_rho1_generic<0, uint8_t, false>), dim3((nw + 3) / 4), dim3(256),
                               0, s, M, D, t->tiles, nw, (const uint8_t *)t->occ_d, t->t1_d,
                               (const double2 *)C_d, part);
    } else {
        if (big)
            hipLaunchKernelGGL((k_rho1_generic<0, uint16_t, true>), dim3((nw + 3) / 4), dim3(256),
                               0, s, M, D, t->tiles, nw, (const uint16_t *)t->occ_d, t->t1_d,
                               (const double2 *)C_d, part);
        else
            hipLaunchKernelGGL((k_rho1_generic<0, uint16_t, false>), dim3((nw + 3) / 4),
                               dim3(256), 0, s, M, D, t->tiles, nw, (const uint16_t *)t->occ_d,
                               t->t1_d, (const double2 *)C_d, part);
    }
    // element e = k M + l, summed over waves by the fixed tree
    hipLaunchKernelGGL(k_gram_sum, dim3(M * M), dim3(256), 0, s, nw, part, (double2 *)rho1_d);
    return launch_status();
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

int mc_zgemv_n(int32_t K, int64_t n, const double *V_d, int64_t ldv, const double *c_d,
               double *out_d, mc_stream stream)
{
    if (K < 1 || n < 0 || ldv < n) return MC_EINVAL;
    if (n == 0) return MC_OK;
    if (!V_d || !out_d || !c_d) return MC_EINVAL;
    if (overlaps(V_d, (size_t)((K - 1) * ldv + n) * 16, out_d, (size_t)n * 16)) return MC_EINVAL;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_zgemv_n, dim3(blocks), dim3(256), 0, (hipStream_t)stream, K, n,
                       (const double2 *)V_d, ldv, (const double2 *)c_d, (double2 *)out_d);
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

int mc_apply_stream_columns(int32_t M, int32_t form, int32_t *slots, int32_t *table_columns)
{
    if (!slots || !table_columns || M < 1 || M > 8) return MC_EINVAL;
    if (form != MC_FORM_PAPER && form != MC_FORM_REDUCED) return MC_EINVAL;
    const bool paper = form == MC_FORM_PAPER;
    *slots = M * (M - 1) + (paper ? M * (M + 1) / 2 * M * M
                                  : M * reduced_slots(M, 0, 0) +
                                        (M * (M - 1) / 2) * (M >= 2 ? reduced_slots(M, 0, 1) : 0));
    *table_columns = *slots;
    switch (M) {
    case 2: *table_columns = paper ? kClassPlan<2, 1>.anchors : kClassPlan<2, 0>.anchors; break;
    case 3: *table_columns = paper ? kClassPlan<3, 1>.anchors : kClassPlan<3, 0>.anchors; break;
    case 4: *table_columns = paper ? kClassPlan<4, 1>.anchors : kClassPlan<4, 0>.anchors; break;
    case 5: *table_columns = paper ? kClassPlan<5, 1>.anchors : kClassPlan<5, 0>.anchors; break;
    case 6:
        if (paper ? kStreamMaxMPaper >= 6 : kStreamMaxMReduced >= 6)
            *table_columns = paper ? kClassPlan<6, 1>.anchors : kClassPlan<6, 0>.anchors;
        break;
    case 7:
        if (!paper && kStreamMaxMReduced >= 7) *table_columns = kClassPlan<7, 0>.anchors;
        break;
    default: break;
    }
    return MC_OK;
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
    case MC_OP_APPLY: {
        // staged constants of either form (plus the sparse lists of the
        // case-split form)
        const int64_t paper = (P * M * M + M * M) * 16;
        const int64_t split = M <= 8 ? split_total(M) * 16 + kSlInts * 4 : 0;
        *bytes = (size_t)(paper > split ? paper : split);
        return MC_OK;
    }
    case MC_OP_RHO1:
        *bytes = M > 8 ? (size_t)rho_waves(tiles) * M * M * 16 : gram_table_workspace(N, M, 1);
        return *bytes ? MC_OK : MC_ERANGE;
    case MC_OP_RHO2:
        *bytes = M > 8 ? 16 : gram_table_workspace(N, M, 2);
        return *bytes ? MC_OK : MC_ERANGE;
    case MC_OP_DOT: *bytes = (size_t)(MC_DOT_BLOCKS + 1) * 16; return MC_OK;
    case MC_OP_RHO1_DIRECT: *bytes = gram_workspace(N, M, 1); return *bytes ? MC_OK : MC_ERANGE;
    case MC_OP_RHO2_DIRECT: *bytes = gram_workspace(N, M, 2); return *bytes ? MC_OK : MC_ERANGE;
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
    if (t->form == MC_FORM_REDUCED) {
        if (M > 8) return MC_EINVAL;
        const size_t sqb = (size_t)(N + 3) * 8;
        if (sqb > 65536) return MC_EINVAL;
        double2 *cf = (double2 *)ws_d;
        hipLaunchKernelGGL(k_prep_split, dim3(4), dim3(256), 0, s, M, adjoint,
                           (const double2 *)g_d, (const double2 *)h_d, cf);
        const int64_t nblocks = (t->tiles + 3) / 4;
        const bool big = D * 16 > (int64_t)0xFFFFFFFFu;
        bool launched = false;
        // same instantiation rules as the paper form: 16-bit occupations only
        // for M <= 5, 64-bit gathers only without a map
#define MC_SPLIT_LAUNCH(OT, BIG, MAP)                                                          \
    MC_DISPATCH_M(M, if constexpr (MT > 0 && (MT <= 5 || sizeof(OT) == 1) && !(BIG && MAP)) {   \
        hipLaunchKernelGGL((k_apply_split<MT, OT, BIG, MAP>), dim3(nblocks), dim3(256),         \
                           kLdsRoots<MT> ? sqb : 0, s, N, D, t->tiles, nblocks, t->t2_entries,   \
                           (const OT *)t->occ_d, t->t1_d, t->pmask_d, t->t2_off_d, t->t2_d,     \
                           (const double2 *)cf, (const double2 *)C_d, (double2 *)HC_d);         \
        launched = true;                                                                       \
    })
        if (chained) {
            if (occ_width(N) == 1) {
                if (big) { MC_SPLIT_LAUNCH(uint8_t, true, false); } else { MC_SPLIT_LAUNCH(uint8_t, false, false); }
            } else {
                if (big) { MC_SPLIT_LAUNCH(uint16_t, true, false); } else { MC_SPLIT_LAUNCH(uint16_t, false, false); }
            }
        } else if (!big) {
            if (occ_width(N) == 1) { MC_SPLIT_LAUNCH(uint8_t, false, true); } else { MC_SPLIT_LAUNCH(uint16_t, false, true); }
        }
#undef MC_SPLIT_LAUNCH
        if (!launched) return MC_EINVAL;
        return launch_status();
    }
    double2 *gp = (double2 *)ws_d;
    double2 *hp = gp + (size_t)npairs(M) * M * M;
    hipLaunchKernelGGL(k_prep, dim3(4), dim3(256), 0, s, M, adjoint, (const double2 *)g_d,
                       (const double2 *)h_d, gp, hp);
    const int64_t nblocks = (t->tiles + 3) / 4;
    const bool big = D * 16 > (int64_t)0xFFFFFFFFu;
    const size_t sqb = (size_t)(N + 3) * 8;   // LDS square-root table (kLdsRoots)
    if (sqb > 65536) return MC_EINVAL;
    // Instantiated combinations: 16-bit occupations only for M <= 5 (M >= 6
    // with N > 255 has D > 2^31), 64-bit gathers (D >= 2^28) only without the
    // double-jump map (a double-jump map of that size cannot fit in HBM).
    bool launched = false;
#define MC_APPLY_LAUNCH(OT, BIG)                                                               \
    if (M <= 8) {                                                                              \
        MC_DISPATCH_M(M, if constexpr (MT > 0 && !BIG && (MT <= 5 || sizeof(OT) == 1)) {        \
            hipLaunchKernelGGL((k_apply<MT, OT, BIG>), dim3(nblocks), dim3(256),                \
                               kLdsRoots<MT> ? sqb : 0, s, N, D,                               \
                               t->tiles, nblocks, t->t2_entries, (const OT *)t->occ_d, t->t1_d,  \
                               t->pmask_d, t->t2_off_d, t->t2_d, (const double2 *)hp,            \
                               (const double2 *)gp, (const double2 *)C_d, (double2 *)HC_d);     \
            launched = true;                                                                   \
        });                                                                                    \
    } else {                                                                                   \
        hipLaunchKernelGGL((k_apply_generic<OT, BIG>), dim3(t->tiles), dim3(64),                \
                           (size_t)5 * M * kTile * 8, s, M, D, t->tiles, t->t2_entries,        \
                           (const OT *)t->occ_d, t->t1_d, t->pmask_d, t->t2_off_d, t->t2_d,    \
                           (const double2 *)hp, (const double2 *)gp, (const double2 *)C_d,     \
                           (double2 *)HC_d);                                                   \
        launched = true;                                                                       \
    }
#define MC_CHAINED_LAUNCH(OT, BIG)                                                             \
    MC_DISPATCH_M(M, if constexpr (MT > 0 && (MT <= 5 || sizeof(OT) == 1)) {                     \
        hipLaunchKernelGGL((k_apply_chained<MT, OT, BIG>), dim3(nblocks), dim3(256),            \
                           kLdsRoots<MT> ? sqb : 0, s, N, D,                                     \
                           t->tiles, nblocks, (const OT *)t->occ_d, t->t1_d, (const double2 *)hp, \
                           (const double2 *)gp, (const double2 *)C_d, (double2 *)HC_d);         \
        launched = true;                                                                       \
    })
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
#undef MC_APPLY_LAUNCH
    if (!launched) return MC_EINVAL;
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

int mc_apply_H_sparse(int32_t N, int32_t M, const double *h_d, const double *g_d,
                      const mc_tables *t, const double *C_d, double *HC_d, void *ws_d,
                      size_t ws_bytes, mc_stream stream)
{
    int st = check_nm(N, M);
    if (st) return st;
    if (!t) return MC_EINVAL;
    const bool chained = t->t2_d == nullptr;
    st = check_tables(N, M, t, !chained);
    if (st) return st;
    if (t->form != MC_FORM_REDUCED || M > 8) return MC_EINVAL;
    if (!h_d || !g_d || !C_d || !HC_d || !ws_d) return MC_EINVAL;
    const int64_t D = t->dim;
    if (overlaps(C_d, (size_t)D * 16, HC_d, (size_t)D * 16)) return MC_EINVAL;
    size_t need = 0;
    mc_workspace_size(N, M, MC_OP_APPLY, &need);
    if (ws_bytes < need) return MC_ENOMEM;
    const size_t sqb = (size_t)(N + 3) * 8;
    if (sqb > 65536) return MC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    double2 *cf = (double2 *)ws_d;
    int32_t *sl = (int32_t *)(cf + split_total(M));
    hipLaunchKernelGGL(k_prep_split, dim3(4), dim3(256), 0, s, M, 0, (const double2 *)g_d,
                       (const double2 *)h_d, cf);
    hipLaunchKernelGGL(k_sparse_lists, dim3(1), dim3(64), 0, s, M, (const double2 *)cf, sl);
    const int64_t nblocks = (t->tiles + 3) / 4;
    const bool big = D * 16 > (int64_t)0xFFFFFFFFu;
    bool launched = false;
#define MC_SPARSE_LAUNCH(OT, BIG, MAP)                                                         \
    MC_DISPATCH_M(M, if constexpr (MT > 0 && (MT <= 5 || sizeof(OT) == 1) && !(BIG && MAP)) {   \
        hipLaunchKernelGGL((k_apply_sparse<MT, OT, BIG, MAP>), dim3(nblocks), dim3(256), sqb, s, \
                           N, D, t->tiles, nblocks, t->t2_entries, (const OT *)t->occ_d,         \
                           t->t1_d, t->pmask_d, t->t2_off_d, t->t2_d, (const double2 *)cf,       \
                           (const int32_t *)sl, (const double2 *)C_d, (double2 *)HC_d);         \
        launched = true;                                                                       \
    })
    if (chained) {
        if (occ_width(N) == 1) {
            if (big) { MC_SPARSE_LAUNCH(uint8_t, true, false); } else { MC_SPARSE_LAUNCH(uint8_t, false, false); }
        } else {
            if (big) { MC_SPARSE_LAUNCH(uint16_t, true, false); } else { MC_SPARSE_LAUNCH(uint16_t, false, false); }
        }
    } else if (!big) {
        if (occ_width(N) == 1) { MC_SPARSE_LAUNCH(uint8_t, false, true); } else { MC_SPARSE_LAUNCH(uint16_t, false, true); }
    }
#undef MC_SPARSE_LAUNCH
    if (!launched) return MC_EINVAL;
    return launch_status();
}

// Scratch of mc_apply_H_direct_noalloc: the staged constants of the apply
// live in this file-scope device array (one copy per GPU, held until the
// process ends) instead of a caller workspace.  Host code never passes the
// array's name to a kernel: its device address is looked up once per device
// (with that device current) and kept per device.
static __device__ __align__(256) unsigned char scratch[MC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static int noalloc_scratch(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_hip_error(e);
    if (dev < 0 || dev >= kMaxDevices) return MC_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return set_hip_error(e != hipSuccess ? e : hipErrorUnknown);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MC_OK;
}

static int apply_direct_common(int32_t N, int32_t M, const double *h_d, const double *g_d,
                               const double *C_d, double *HC_d, void *ws_d, size_t ws_bytes,
                               int adjoint, mc_stream stream)
{
    int st = check_nm(N, M);
    if (st) return st;
    if (M > 8) return MC_EINVAL;
    const int64_t D = dim_checked(N, M);
    if (D < 0 || D >= ((int64_t)1 << 31)) return MC_ERANGE;
    if (!h_d || !g_d || !C_d || !HC_d || !ws_d) return MC_EINVAL;
    if (overlaps(C_d, (size_t)D * 16, HC_d, (size_t)D * 16)) return MC_EINVAL;
    size_t need = 0;
    mc_workspace_size(N, M, MC_OP_APPLY, &need);
    if (ws_bytes < need) return MC_ENOMEM;
    const size_t sqb = (size_t)(N + 3) * 8;
    if (M >= MC_LDS_ROOTS_FROM && sqb > 65536) return MC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    double2 *cf = (double2 *)ws_d;
    hipLaunchKernelGGL(k_prep_split, dim3(4), dim3(256), 0, s, M, adjoint, (const double2 *)g_d,
                       (const double2 *)h_d, cf);
    const int64_t tiles = (D + kTile - 1) / kTile;
    const int64_t nblocks = (tiles + 3) / 4;
    const int nbits = bit_width(N);
    const bool big = D * 16 > (int64_t)0xFFFFFFFFu;
    MC_DISPATCH_M(M, if constexpr (MT > 0 && MT <= 8) {
        if (big)
            hipLaunchKernelGGL((k_apply_direct<MT, true>), dim3(nblocks), dim3(256),
                               kLdsRoots<MT> ? sqb : 0, s, N, nbits, D, tiles, nblocks,
                               (const double2 *)cf, (const double2 *)C_d, (double2 *)HC_d);
        else
            hipLaunchKernelGGL((k_apply_direct<MT, false>), dim3(nblocks), dim3(256),
                               kLdsRoots<MT> ? sqb : 0, s, N, nbits, D, tiles, nblocks,
                               (const double2 *)cf, (const double2 *)C_d, (double2 *)HC_d);
    });
    return launch_status();
}

int mc_apply_H_direct(int32_t N, int32_t M, const double *h_d, const double *g_d,
                      const double *C_d, double *HC_d, void *ws_d, size_t ws_bytes,
                      mc_stream stream)
{
    return apply_direct_common(N, M, h_d, g_d, C_d, HC_d, ws_d, ws_bytes, 0, stream);
}

int mc_apply_H_direct_noalloc(int32_t N, int32_t M, const double *h_d, const double *g_d,
                              const double *C_d, double *HC_d, mc_stream stream)
{
    size_t need = 0;
    int st = mc_workspace_size(N, M, MC_OP_APPLY, &need);
    if (st) return st;
    if (need > (size_t)MC_NOALLOC_SCRATCH_BYTES) return MC_ENOMEM;
    void *ws = nullptr;
    st = noalloc_scratch(&ws);
    if (st) return st;
    return apply_direct_common(N, M, h_d, g_d, C_d, HC_d, ws, MC_NOALLOC_SCRATCH_BYTES, 0,
                               stream);
}

int mc_apply_H_direct_adjoint(int32_t N, int32_t M, const double *h_d, const double *g_d,
                              const double *C_d, double *HC_d, void *ws_d, size_t ws_bytes,
                              mc_stream stream)
{
    return apply_direct_common(N, M, h_d, g_d, C_d, HC_d, ws_d, ws_bytes, 1, stream);
}

int mc_is_hermitian(int32_t M, const double *h_d, const double *g_d, int32_t *flag_d,
                    mc_stream stream)
{
    if (M < 1 || M > MC_MAX_M || !h_d || !g_d || !flag_d) return MC_EINVAL;
    hipLaunchKernelGGL(k_is_hermitian, dim3(1), dim3(256), 0, (hipStream_t)stream, M,
                       (const double2 *)h_d, (const double2 *)g_d, flag_d);
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
