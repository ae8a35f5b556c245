// H.C in the case-split form for interactions with many vanishing
// coefficients (momentum-conserving plane-wave g, lattice models).  After the
// case-split constants are staged, k_sparse_lists compacts the single jumps
// and the reduced double-jump slots whose constants are not all zero into
// lists; the tile walks only those (the row's own term is always taken).
// Entries are wave-uniform, orbitals run-time; the roots come from the
// block's sqrt table.
#pragma once

#include "mc_split.h"

namespace mc {

// List layout (int32, in the workspace after the staged constants):
//   [0]                    number of active single jumps
//   [kSlSingles + i]       active single jump j = a*M + b
//   [kSlPairs + 2p]        first entry of pair p, [kSlPairs + 2p + 1] count
//   [kSlEntries + e]       r | q << 8 | l << 16  (reduced slot r of its pair)
constexpr int kSlSingles = 1;
constexpr int kSlPairs = kSlSingles + 64;
constexpr int kSlEntries = kSlPairs + 2 * 36;
constexpr int kSlInts = kSlEntries + 8 * 28 + 28 * 21;   // M <= 8

__device__ __forceinline__ bool nonzero(double2 v) { return v.x != 0.0 || v.y != 0.0; }

// One thread builds the lists from the staged constants cf (layout of
// mc_split.h).  Run after k_prep_split, before the apply.
__global__ void k_sparse_lists(int M, const double2 *__restrict__ cf, int32_t *__restrict__ sl)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const double2 *HS = cf + split_hs_offset(M), *GS = cf + split_gs_offset(M);
    const double2 *GD = cf + split_gd_offset(M);
    int ns = 0;
    for (int j = 0; j < M * M; ++j) {
        if (j / M == j % M) continue;
        bool any = nonzero(HS[j]);
        for (int c = 0; c < M; ++c) any = any || nonzero(GS[j * M + c]);
        if (any) sl[kSlSingles + ns++] = j;
    }
    sl[0] = ns;
    int p = 0, e = 0, co = 0;
    for (int k = 0; k < M; ++k) {
        for (int s = k; s < M; ++s, ++p) {
            sl[kSlPairs + 2 * p] = e;
            int r = 0;
            for (int q = 0; q < M; ++q) {
                for (int l = q; l < M; ++l) {
                    if (q == k || q == s || l == k || l == s) continue;
                    if (nonzero(GD[co + r])) sl[kSlEntries + e++] = r | (q << 8) | (l << 16);
                    ++r;
                }
            }
            co += r;
            sl[kSlPairs + 2 * p + 1] = e - sl[kSlPairs + 2 * p];
        }
    }
}

template <int MT>
__device__ __forceinline__ int occ_at(const int (&n)[MT], int m)
{
    int v = 0;
#pragma unroll
    for (int i = 0; i < MT; ++i) v = i == m ? n[i] : v;
    return v;
}

#ifndef MC_SPARSE_BATCH
#define MC_SPARSE_BATCH 8
#endif

template <int MT, typename OccT, bool BIGC, bool MAP>
__device__ __forceinline__ void apply_tile_sparse(int64_t tile, int64_t D, int64_t cap,
                                                  const double *sq,
                                                  const OccT *__restrict__ occ,
                                                  const int32_t *__restrict__ t1,
                                                  const uint64_t *__restrict__ pmask,
                                                  const int64_t *__restrict__ t2_off,
                                                  const int32_t *__restrict__ t2r,
                                                  const double2 *__restrict__ cf,
                                                  const int32_t *__restrict__ sl,
                                                  const double2 *__restrict__ C,
                                                  double2 *__restrict__ HC)
{
    constexpr int M = MT;
    constexpr int NP = M * (M + 1) / 2;
    constexpr int W = (NP + 63) / 64;
    constexpr int NS = M * M, SB = MC_SPARSE_BATCH;
    const int lane = threadIdx.x & 63;
    const int64_t g = tile * kTile + lane;
    const bool live = g < D;
    int n[M];
    double x[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        n[m] = (int)occ[(tile * M + m) * kTile + lane];
        x[m] = (double)n[m];
    }
    const Gather<BIGC> ldc(C, D);
    const double2 *DL = cf + split_dl_offset(M), *GI = cf + split_gi_offset(M);
    const double2 *HS = cf + split_hs_offset(M), *GS = cf + split_gs_offset(M);
    const double2 *GD = cf + split_gd_offset(M);

    // the row's own coefficient
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
        for (int p = 0; p < NP; ++p) {
            const double w = x[pair_k(M, p)] * x[pair_s(M, p)];
            dr = fma(GI[p].x, w, dr);
            di = fma(GI[p].y, w, di);
        }
        ar = dr * cg.x - di * cg.y;
        ai = dr * cg.y + di * cg.x;
    }
    const __amdgpu_buffer_rsrc_t r1 = make_rsrc(t1 + tile * NS * kTile, (uint32_t)(NS * kTile * 4));

    // active single jumps
    const int ns = sl[0];
#pragma unroll 1
    for (int i0 = 0; i0 < ns; i0 += SB) {
        int jj[SB];
        int32_t t[SB];
        double2 c[SB];
#pragma unroll
        for (int i = 0; i < SB; ++i) {
            jj[i] = i0 + i < ns ? sl[kSlSingles + i0 + i] : -1;
            t[i] = jj[i] >= 0 ? buf_ld_i32(r1, (uint32_t)((jj[i] * kTile + lane) * 4), 0) : -1;
        }
#pragma unroll
        for (int i = 0; i < SB; ++i) c[i] = ldc(t[i]);
#pragma unroll
        for (int i = 0; i < SB; ++i) {
            const int j = jj[i];
            if (j < 0) break;
            const int a = j / M, b = j % M;
            double er = HS[j].x, ei = HS[j].y;
#pragma unroll
            for (int k = 0; k < M; ++k) {
                er = fma(GS[j * M + k].x, x[k], er);
                ei = fma(GS[j * M + k].y, x[k], ei);
            }
            const double f = sq[occ_at(n, a)] * sq[occ_at(n, b) + 1];
            er *= f;
            ei *= f;
            ar = fma(er, c[i].x, ar);
            ar = fma(-ei, c[i].y, ar);
            ai = fma(er, c[i].y, ai);
            ai = fma(ei, c[i].x, ai);
        }
    }

    // active true double jumps
    int64_t off0 = 0, off1 = 0;
    if constexpr (MAP) t2_block(t2_off, tile, cap, off0, off1);
    const uint64_t *pm = pmask + tile * W;
    int64_t pos = off0;
    int p = 0, co = 0;
#pragma unroll 1
    for (int K = 0; K < M; ++K) {
#pragma unroll 1
        for (int S = K; S < M; ++S, ++p) {
            const int ND = reduced_slots(M, K, S);
            const int cbase = co;
            co += ND;
            __amdgpu_buffer_rsrc_t r2;
            if constexpr (MAP) {
                if (ND == 0 || !((pm[p >> 6] >> (p & 63)) & 1) ||
                    pos + (int64_t)ND * kTile > off1)
                    continue;
                r2 = make_rsrc(t2r + pos, (uint32_t)(ND * kTile * 4));
                pos += (int64_t)ND * kTile;
            }
            const int first = sl[kSlPairs + 2 * p], cnt = sl[kSlPairs + 2 * p + 1];
            if (cnt == 0) continue;
            const int nK = occ_at(n, K), nS = occ_at(n, S);
            const bool valid = K == S ? nK >= 2 : (nK >= 1 && nS >= 1);
            if (!__ballot(valid)) continue;
            const double A = valid ? sq[nK] * (K == S ? sq[nK > 0 ? nK - 1 : 0] : sq[nS]) : 0.0;
            double br = 0.0, bi = 0.0;
#pragma unroll 1
            for (int i0 = 0; i0 < cnt; i0 += SB) {
                int ent[SB];
                int32_t t[SB];
                double2 c[SB];
#pragma unroll
                for (int i = 0; i < SB; ++i) {
                    ent[i] = i0 + i < cnt ? sl[kSlEntries + first + i0 + i] : -1;
                    int32_t v = -1;
                    if (ent[i] >= 0) {
                        const int r = ent[i] & 255, q = (ent[i] >> 8) & 255, l = (ent[i] >> 16) & 255;
                        if constexpr (MAP) {
                            v = buf_ld_i32(r2, (uint32_t)((r * kTile + lane) * 4), 0);
                        } else {
                            const int32_t b =
                                buf_ld_i32(r1, (uint32_t)(((K * M + q) * kTile + lane) * 4), 0);
                            const bool ok = valid && b >= 0 && b < D;
                            const int64_t bb = ok ? b : 0;
                            const int32_t w = t1[((bb >> 6) * NS + S * M + l) * kTile + (bb & 63)];
                            v = ok ? w : -1;
                        }
                    }
                    t[i] = v;
                }
#pragma unroll
                for (int i = 0; i < SB; ++i) c[i] = ldc(t[i]);
#pragma unroll
                for (int i = 0; i < SB; ++i) {
                    if (ent[i] < 0) break;
                    const int r = ent[i] & 255, q = (ent[i] >> 8) & 255, l = (ent[i] >> 16) & 255;
                    const int nq = occ_at(n, q), nl = occ_at(n, l);
                    const double Bf = q == l ? sq[nq + 1] * sq[nq + 2] : sq[nq + 1] * sq[nl + 1];
                    const double2 Gv = GD[cbase + r];
                    const double cr = c[i].x * Bf, ci = c[i].y * Bf;
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
    if (live) HC[g] = make_double2(ar, ai);
}

}  // namespace mc
