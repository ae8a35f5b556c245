// Batched H.C over many (N, M, h, g) instances of uneven size, and the
// segmented vector operations a batched Lanczos recurrence needs.
//
// A batch vector is the concatenation of the instances' coefficient vectors
// (instance i at offset vec_off[i]).  The plan, built once into a caller
// buffer, holds per-instance descriptors and staged coefficients, the
// instances grouped by orbital count, and a chunk table for segmented
// reductions.  Each group runs as one persistent kernel: its wavefronts walk
// the group's (instance, tile) work list, so instances of 45 rows and of
// 6*10^7 rows share the same launch.  Every call only enqueues kernels (no
// host synchronisation, no memset), so a sequence of calls can be captured
// into a HIP graph and replayed.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "mc_apply.h"
#include "mc_split.h"
#include "mc_direct.h"
#include "mc_internal.h"

namespace mc {

// How an instance's tile body runs: paper form through its map or chained,
// case-split form through its reduced map or chained.
enum BatchKind : int32_t { kPaperMap = 0, kPaperChain = 1, kSplitMap = 2, kSplitChain = 3, kDirect = 4 };

struct BatchInst {
    int32_t N, M;
    int32_t kind, nbits;  // nbits: bit width of N (table-free kind)
    int64_t dim, tiles, cap, vec_off;
    const uint8_t *occ;
    const int32_t *t1;
    const uint64_t *pmask;
    const int64_t *t2_off;
    const int32_t *t2;   // null: chain single jumps
    const double2 *h, *g;
    double2 *hp, *gp;    // staged h' and G' (paper form) / gp: case-split constants
    int64_t hp_off, gp_off;  // the same, as offsets into the plan's coefficient region
};

// Pointers read from a descriptor are generic (flat loads); the staged
// constants are therefore reached through the __restrict__ coefficient-region
// kernel argument, which keeps their loads scalar.

// Staged complex constants per instance, enough for either form.
inline int64_t batch_coef_elems(int M)
{
    const int64_t paper = (int64_t)npairs(M) * M * M + (int64_t)M * M;
    const int64_t split = split_total(M);
    return paper > split ? paper : split;
}

struct BatchChunk {
    int32_t inst;
    int32_t pad;
    int64_t start, len;   // in batch-vector elements
};

constexpr int64_t kChunk = 1 << 16;
constexpr int kMaxGroups = 40;   // 8 orbital counts x 5 kinds
constexpr int kGrab = 8;         // tiles a wavefront takes per counter increment (order 3)

// An instance launched on a grid of its own; its tables are passed to the
// kernel as arguments (global, non-aliasing: the same loads as mc_apply_H).
struct SoloLaunch {
    int32_t j;      // sorted position (index into the plan's descriptors)
    int32_t M, kind, N;
    int64_t tiles, dim, cap, vec_off, gp_off, hp_off;
    const uint8_t *occ;
    const int32_t *t1;
    const uint64_t *pmask;
    const int64_t *t2_off;
    const int32_t *t2;
};

}  // namespace mc

struct mc_batch {
    int32_t count;
    int32_t ngroups;
    int32_t group_M[40];
    int32_t group_kind[40];   // BatchKind of the group's instances
    int32_t group_first[40];  // first entry in the sorted instance order
    int32_t group_count[40];
    int64_t group_tiles[40];
    int64_t group_blocks[40];
    int64_t nchunks;
    int64_t total_len;        // batch-vector length
    int32_t order;
    mc::BatchInst *inst_d;    // [count], in sorted order
    int64_t *tile_prefix_d;   // [count + 1] per sorted instance, restarting per group
    mc::BatchChunk *chunks_d; // [nchunks]
    double2 *partials_d;      // [nchunks]
    int32_t *sorted_d;        // [count] sorted position -> caller index
    int32_t *pos_d;           // [count] caller index -> sorted position
    uint32_t *counters_d;     // [kMaxGroups] work counters of order 3, zeroed per apply
    double2 *coef_d;          // staged coefficients of all instances
    int32_t nsolo;            // instances launched on grids of their own
    mc::SoloLaunch *solo;     // [nsolo] (host)
};

namespace mc {

__global__ void k_batch_prep(const BatchInst *__restrict__ inst, uint32_t *__restrict__ counters)
{
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < kMaxGroups) counters[threadIdx.x] = 0;
    const BatchInst I = inst[blockIdx.y];
    const int M = I.M;
    const int first = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    if (I.kind == kSplitMap || I.kind == kSplitChain || I.kind == kDirect) {
        stage_split_constants(M, 0, I.g, I.h, I.gp, first, stride);
        return;
    }
    const int P = M * (M + 1) / 2;
    const int total = P * M * M;
    for (int idx = first; idx < total + M * M; idx += stride) {
        if (idx >= total) {
            const int e = idx - total;
            I.hp[e] = I.h[e];
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
        double2 a = I.g[((k * M + s) * M + q) * M + l];
        if (k != s) {
            const double2 b = I.g[((s * M + k) * M + q) * M + l];
            a.x += b.x;
            a.y += b.y;
        }
        I.gp[idx] = make_double2(0.5 * a.x, 0.5 * a.y);
    }
}

// One tile of one instance, in the instance's kind.
template <int MT, int KIND>
__device__ __forceinline__ void batch_tile(const BatchInst &I, int64_t tile, const double *sq,
                                           const double2 *__restrict__ coef,
                                           const double2 *__restrict__ Cb,
                                           double2 *__restrict__ HCb)
{
    const double2 *C = Cb + I.vec_off;
    double2 *HC = HCb + I.vec_off;
    const uint8_t *occ = I.occ;
    const int32_t *t1 = I.t1;
    const uint64_t *pmask = I.pmask;
    const int64_t *t2_off = I.t2_off;
    const int32_t *t2 = I.t2;
    const double2 *gp = coef + I.gp_off, *hp = coef + I.hp_off;
    if constexpr (KIND == kPaperMap)
        apply_tile_paper<MT, uint8_t, false>(tile, I.dim, I.cap, sq, occ, t1, pmask, t2_off, t2, hp,
                                          gp, C, HC);
    else if constexpr (KIND == kPaperChain)
        apply_tile_chained<MT, uint8_t, false>(tile, I.dim, sq, occ, t1, hp, gp, C, HC);
    else if constexpr (KIND == kDirect)
        apply_tile_direct<MT, false>(tile, I.N, I.nbits, I.dim, sq, gp, C, HC);
    else
        apply_tile_split<MT, uint8_t, false, KIND == kSplitMap>(tile, I.dim, I.cap, sq, occ, t1,
                                                                pmask, t2_off, t2, gp, C, HC);
}

// Persistent H.C over one group (one orbital count and one BatchKind).
// Work item i of the group is tile (i - prefix[j]) of the group's j-th
// instance; with order 0 wavefront w takes items w, w + W, w + 2W, ...
// (neighbouring tiles on neighbouring wavefronts), with order 1 a contiguous
// range of items, with order 2 each XCD a contiguous share of the items,
// interleaved over its wavefronts; with order 3 wavefronts take kGrab items
// at a time from a per-group counter (dynamic balance, like a plain launch).
constexpr int kBatchMaxN = 255;

template <int MT, int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MC_APPLY_WAVES)))
void k_batch_apply(const BatchInst *__restrict__ inst, const int64_t *__restrict__ prefix,
                   int first, int count, int64_t items, int64_t nblocks, int order,
                   uint32_t *__restrict__ counter, const double2 *__restrict__ coef,
                   const double2 *__restrict__ Cb, double2 *__restrict__ HCb)
{
    __shared__ double sq[kLdsRoots<MT> ? kBatchMaxN + 3 : 1];
    if constexpr (kLdsRoots<MT>) fill_sqrt_table(sq, kBatchMaxN + 3);
    auto tile_body = [&](int64_t i, int &j) __attribute__((always_inline)) {
        // instance of item i (prefix is non-decreasing; a wavefront visits
        // items in increasing order, so the search resumes where it stopped)
        while (j + 1 < count && prefix[first + j + 1] <= i) ++j;
        const BatchInst I = inst[first + j];
        batch_tile<MT, KIND>(I, i - prefix[first + j], sq, coef, Cb, HCb);
    };
    int j = 0;
    if (order == 3) {
        // dynamic: take kGrab items at a time from the group's counter (a
        // vector atomic from lane 0; the count is zeroed by k_batch_prep)
        for (;;) {
            uint32_t base = 0;
            if ((threadIdx.x & 63) == 0) base = atomicAdd(counter, (uint32_t)kGrab);
            base = __builtin_amdgcn_readfirstlane(base);
            if ((int64_t)base >= items) break;
            const int64_t end = (int64_t)base + kGrab < items ? (int64_t)base + kGrab : items;
            for (int64_t i = base; i < end; ++i) tile_body(i, j);
        }
        return;
    }
    const int64_t W = nblocks * 4;
    const int64_t w = xcd_block(blockIdx.x, nblocks) * 4 + wave_in_block();
    int64_t i0, step, iend;
    if (order == 2) {
        // blocks go to XCD b % 8; this XCD's blocks own items [ib, ie)
        const int64_t xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
        const int64_t bper = nblocks >> 3, brem = nblocks & 7;
        const int64_t nbx = bper + (xcd < brem ? 1 : 0);
        const int64_t fb = xcd * bper + (xcd < brem ? xcd : brem);
        const int64_t ib = items * fb / nblocks, ie = items * (fb + nbx) / nblocks;
        i0 = ib + local * 4 + wave_in_block();
        step = nbx * 4;
        iend = ie;
    } else if (order == 1) {
        const int64_t per = (items + W - 1) / W;
        i0 = w * per;
        step = 1;
        iend = i0 + per < items ? i0 + per : items;
    } else {
        i0 = w;
        step = W;
        iend = items;
    }
    for (int64_t i = i0; i < iend; i += step) tile_body(i, j);
}

// One large instance on a grid of its own: one wavefront per tile, blocks
// remapped per XCD as in the plain apply; tables, staged constants and the
// instance's vector segments arrive as kernel arguments.
template <int MT, int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MC_APPLY_WAVES)))
void k_batch_solo(int N, int nbits, int64_t D, int64_t tiles, int64_t nblocks, int64_t cap,
                  const uint8_t *__restrict__ occ, const int32_t *__restrict__ t1,
                  const uint64_t *__restrict__ pmask, const int64_t *__restrict__ t2_off,
                  const int32_t *__restrict__ t2, const double2 *__restrict__ gp,
                  const double2 *__restrict__ hp, const double2 *__restrict__ C,
                  double2 *__restrict__ HC)
{
    __shared__ double sq[kLdsRoots<MT> ? kBatchMaxN + 3 : 1];
    // one instance: the roots it needs, as the plain launch fills them
    if constexpr (kLdsRoots<MT>) fill_sqrt_table(sq, N + 3 < kBatchMaxN + 3 ? N + 3 : kBatchMaxN + 3);
    const int64_t tile =
        xcd_block_as<KIND == kDirect && kDirectRemap<MT>>(blockIdx.x, nblocks) * 4 + wave_in_block();
    if (tile >= tiles) return;
    if constexpr (KIND == kPaperMap)
        apply_tile_paper<MT, uint8_t, false>(tile, D, cap, sq, occ, t1, pmask, t2_off, t2, hp, gp, C,
                                          HC);
    else if constexpr (KIND == kPaperChain)
        apply_tile_chained<MT, uint8_t, false>(tile, D, sq, occ, t1, hp, gp, C, HC);
    else if constexpr (KIND == kDirect)
        apply_tile_direct<MT, false>(tile, N, nbits, D, sq, gp, C, HC);
    else
        apply_tile_split<MT, uint8_t, false, KIND == kSplitMap>(tile, D, cap, sq, occ, t1, pmask,
                                                                t2_off, t2, gp, C, HC);
}

// Segmented conj(x).y: chunk partials, then per-instance sums in chunk order.
__global__ __launch_bounds__(256) void k_seg_dot_partial(const BatchChunk *__restrict__ ch,
                                                          int64_t nchunks,
                                                          const double2 *__restrict__ x,
                                                          const double2 *__restrict__ y,
                                                          double2 *__restrict__ part)
{
    __shared__ double sr[4], si[4];
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const BatchChunk C = ch[c];
        double ar = 0.0, ai = 0.0;
        for (int64_t i = C.start + threadIdx.x; i < C.start + C.len; i += blockDim.x) {
            const double2 a = x[i], b = y[i];
            ar += a.x * b.x + a.y * b.y;
            ai += a.x * b.y - a.y * b.x;
        }
        ar = wave_sum(ar);
        ai = wave_sum(ai);
        if ((threadIdx.x & 63) == 0) {
            sr[wave_in_block()] = ar;
            si[wave_in_block()] = ai;
        }
        __syncthreads();
        if (threadIdx.x == 0)
            part[c] = make_double2((sr[0] + sr[1]) + (sr[2] + sr[3]), (si[0] + si[1]) + (si[2] + si[3]));
        __syncthreads();
    }
}

// out[caller index] = sum of the instance's chunk partials (chunks of an
// instance are contiguous and in order); sqrt_real: write sqrt(Re) as double.
__global__ void k_seg_final(const BatchChunk *__restrict__ ch, int64_t nchunks, int count,
                            const int32_t *__restrict__ sorted, const double2 *__restrict__ part,
                            double2 *__restrict__ out_c, double *__restrict__ out_norm)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count) return;
    // binary search for the first chunk of sorted instance j
    int64_t lo = 0, hi = nchunks;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (ch[mid].inst < j) lo = mid + 1;
        else hi = mid;
    }
    double sr = 0.0, si = 0.0;
    for (int64_t c = lo; c < nchunks && ch[c].inst == j; ++c) {
        sr += part[c].x;
        si += part[c].y;
    }
    const int dst = sorted[j];
    if (out_c) out_c[dst] = make_double2(sr, si);
    if (out_norm) out_norm[dst] = sqrt(sr);
}

// w -= Re(alpha_i) v + beta_i v_prev per instance segment (three-term step)
__global__ __launch_bounds__(256) void k_seg_orth(const BatchChunk *__restrict__ ch,
                                                   int64_t nchunks,
                                                   const int32_t *__restrict__ sorted,
                                                   double2 *__restrict__ w,
                                                   const double2 *__restrict__ v,
                                                   const double2 *__restrict__ vp,
                                                   const double2 *__restrict__ alpha,
                                                   const double *__restrict__ beta)
{
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const BatchChunk C = ch[c];
        const int dst = sorted[C.inst];
        const double a = alpha[dst].x;
        const double b = (vp && beta) ? beta[dst] : 0.0;
        for (int64_t i = C.start + threadIdx.x; i < C.start + C.len; i += blockDim.x) {
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
}

// out = w / beta_i per instance segment (0 where beta_i = 0)
__global__ __launch_bounds__(256) void k_seg_scale(const BatchChunk *__restrict__ ch,
                                                    int64_t nchunks,
                                                    const int32_t *__restrict__ sorted,
                                                    const double2 *__restrict__ w,
                                                    const double *__restrict__ beta,
                                                    double2 *__restrict__ out)
{
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const BatchChunk C = ch[c];
        const double b = beta[sorted[C.inst]];
        const double inv = b > 0.0 ? 1.0 / b : 0.0;
        for (int64_t i = C.start + threadIdx.x; i < C.start + C.len; i += blockDim.x) {
            const double2 x = w[i];
            out[i] = make_double2(x.x * inv, x.y * inv);
        }
    }
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct PlanLayout {
    size_t inst, prefix, chunks, partials, sorted, pos, counters, coef, total;
};

// An item whose descriptor holds sizes but no buffers runs table-free.
static bool table_free(const mc_tables *t)
{
    return !t->binom_d && !t->occ_d && !t->t1_d && !t->pmask_d && !t->t2_off_d && !t->t2_d;
}

static int plan_layout(int32_t count, const mc_batch_item *items, int64_t *nchunks_out,
                       int64_t *coef_elems_out, PlanLayout *L)
{
    int64_t nchunks = 0, coef = 0;
    for (int i = 0; i < count; ++i) {
        const mc_tables *t = items[i].tables;
        if (!t) return MC_EINVAL;
        const int M = t->M;
        nchunks += (t->dim + kChunk - 1) / kChunk;
        coef += batch_coef_elems(M);
    }
    L->inst = 0;
    L->prefix = align256(L->inst + sizeof(BatchInst) * count);
    L->chunks = align256(L->prefix + sizeof(int64_t) * (count + 1));
    L->partials = align256(L->chunks + sizeof(BatchChunk) * nchunks);
    L->sorted = align256(L->partials + sizeof(double2) * nchunks);
    L->pos = align256(L->sorted + sizeof(int32_t) * count);
    L->counters = align256(L->pos + sizeof(int32_t) * count);
    L->coef = align256(L->counters + sizeof(uint32_t) * kMaxGroups);
    L->total = align256(L->coef + sizeof(double2) * coef);
    *nchunks_out = nchunks;
    *coef_elems_out = coef;
    return MC_OK;
}

}  // namespace mc

using namespace mc;

extern "C" {

int mc_batch_plan_size(int32_t count, const mc_batch_item *items, size_t *bytes)
{
    if (count < 1 || !items || !bytes) return MC_EINVAL;
    PlanLayout L;
    int64_t nch, coef;
    const int st = plan_layout(count, items, &nch, &coef, &L);
    if (st) return st;
    *bytes = L.total;
    return MC_OK;
}

int mc_batch_create(int32_t count, const mc_batch_item *items, const mc_batch_schedule *sched,
                    void *plan_d, size_t plan_bytes, mc_stream stream, mc_batch **out)
{
    if (count < 1 || !items || !out || !plan_d) return MC_EINVAL;
    *out = nullptr;
    for (int i = 0; i < count; ++i) {
        const mc_tables *t = items[i].tables;
        if (!t || !items[i].h_d || !items[i].g_d) return MC_EINVAL;
        int st = check_nm(t->N, t->M);
        if (st) return st;
        if (table_free(t)) {
            // sizes only: they must be those of (N, M)
            const int64_t D = dim_checked(t->N, t->M);
            if (D < 0 || t->dim != D || t->tiles != (D + kTile - 1) / kTile) return MC_EINVAL;
        } else {
            st = check_tables(t->N, t->M, t, t->t2_d != nullptr);
            if (st) return st;
        }
        // batched instances: M <= 8, N <= 255, D < 2^28 (range-checked gathers)
        if (t->M > 8 || occ_width(t->N) != 1 || t->dim * 16 > (int64_t)0xFFFFFFFFu) return MC_EINVAL;
    }
    PlanLayout L;
    int64_t nchunks, coef_elems;
    int st = plan_layout(count, items, &nchunks, &coef_elems, &L);
    if (st) return st;
    if (plan_bytes < L.total) return MC_ENOMEM;
    const int bpc = sched && sched->blocks_per_cu > 0 ? sched->blocks_per_cu : 2;
    const int order = sched ? sched->order : 0;
    if (order < 0 || order > 3) return MC_EINVAL;

    // instance order: by orbital count, then kind, then decreasing dimension
    auto kind_of = [](const mc_tables *t) -> int32_t {
        if (table_free(t)) return kDirect;
        const bool split = t->form == MC_FORM_REDUCED, map = t->t2_d != nullptr;
        return split ? (map ? kSplitMap : kSplitChain) : (map ? kPaperMap : kPaperChain);
    };
    std::vector<int32_t> sorted(count);
    std::iota(sorted.begin(), sorted.end(), 0);
    std::stable_sort(sorted.begin(), sorted.end(), [&](int a, int b) {
        const mc_tables *x = items[a].tables, *y = items[b].tables;
        if (x->M != y->M) return x->M < y->M;
        if (kind_of(x) != kind_of(y)) return kind_of(x) < kind_of(y);
        return x->dim > y->dim;
    });
    mc_batch *b = (mc_batch *)calloc(1, sizeof(mc_batch));
    if (!b) return MC_ENOMEM;
    b->solo = (SoloLaunch *)calloc((size_t)count, sizeof(SoloLaunch));
    if (!b->solo) {
        free(b);
        return MC_ENOMEM;
    }
    const int64_t solo_min = sched && sched->solo_tiles > 0 ? sched->solo_tiles : 0;
    b->count = count;
    b->order = order;
    std::vector<int32_t> pos(count);
    std::vector<BatchInst> inst(count);
    std::vector<int64_t> prefix(count + 1, 0);
    std::vector<BatchChunk> chunks;
    chunks.reserve(nchunks);
    char *base = (char *)plan_d;
    double2 *coef = (double2 *)(base + L.coef);
    int64_t voff = 0, cpos = 0;
    for (int j = 0; j < count; ++j) {
        const int i = sorted[j];
        pos[i] = j;
        const mc_tables *t = items[i].tables;
        BatchInst &I = inst[j];
        I.N = t->N;
        I.M = t->M;
        I.kind = kind_of(t);
        I.nbits = bit_width(t->N);
        I.dim = t->dim;
        I.tiles = t->tiles;
        I.cap = t->t2_d ? t->t2_entries : 0;
        I.vec_off = 0;
        I.occ = (const uint8_t *)t->occ_d;
        I.t1 = t->t1_d;
        I.pmask = t->pmask_d;
        I.t2_off = t->t2_off_d;
        I.t2 = t->t2_d;
        I.h = (const double2 *)items[i].h_d;
        I.g = (const double2 *)items[i].g_d;
        I.gp = coef + cpos;
        I.hp = coef + cpos + (int64_t)npairs(t->M) * t->M * t->M;
        I.gp_off = cpos;
        I.hp_off = cpos + (int64_t)npairs(t->M) * t->M * t->M;
        cpos += batch_coef_elems(t->M);
        // a large instance gets a launch of its own; the rest join groups
        if (solo_min > 0 && t->tiles >= solo_min) {
            SoloLaunch &L1 = b->solo[b->nsolo++];
            L1.j = j;
            L1.M = t->M;
            L1.kind = I.kind;
            L1.N = t->N;
            L1.tiles = t->tiles;
            L1.dim = t->dim;
            L1.cap = I.cap;
            L1.gp_off = I.gp_off;
            L1.hp_off = I.hp_off;
            L1.occ = I.occ;
            L1.t1 = I.t1;
            L1.pmask = I.pmask;
            L1.t2_off = I.t2_off;
            L1.t2 = I.t2;
            prefix[j] = 0;
            continue;
        }
        // group bookkeeping
        if (b->ngroups == 0 || b->group_M[b->ngroups - 1] != t->M ||
            b->group_kind[b->ngroups - 1] != I.kind) {
            b->group_M[b->ngroups] = t->M;
            b->group_kind[b->ngroups] = I.kind;
            b->group_first[b->ngroups] = j;
            b->group_count[b->ngroups] = 0;
            b->group_tiles[b->ngroups] = 0;
            ++b->ngroups;
        }
        const int gi = b->ngroups - 1;
        prefix[j] = b->group_tiles[gi];
        b->group_tiles[gi] += t->tiles;
        ++b->group_count[gi];
    }
    // vector offsets follow the caller's order so that batch vectors are laid
    // out instance by instance as the caller listed them
    {
        std::vector<int64_t> off(count);
        for (int i = 0; i < count; ++i) {
            off[i] = voff;
            voff += items[i].tables->dim;
        }
        for (int j = 0; j < count; ++j) inst[j].vec_off = off[sorted[j]];
        for (int k = 0; k < b->nsolo; ++k) b->solo[k].vec_off = inst[b->solo[k].j].vec_off;
        for (int j = 0; j < count; ++j) {
            const int64_t D = inst[j].dim;
            for (int64_t s = 0; s < D; s += kChunk) {
                BatchChunk c;
                c.inst = j;
                c.pad = 0;
                c.start = inst[j].vec_off + s;
                c.len = D - s < kChunk ? D - s : kChunk;
                chunks.push_back(c);
            }
        }
    }
    b->total_len = voff;
    b->nchunks = (int64_t)chunks.size();
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    }
    for (int gi = 0; gi < b->ngroups; ++gi) {
        const int64_t need = (b->group_tiles[gi] + 3) / 4;
        const int64_t cap_blocks = (int64_t)bpc * cus;
        b->group_blocks[gi] = need < cap_blocks ? need : cap_blocks;
        if (b->group_blocks[gi] < 1) b->group_blocks[gi] = 1;
    }
    b->inst_d = (BatchInst *)(base + L.inst);
    b->tile_prefix_d = (int64_t *)(base + L.prefix);
    b->chunks_d = (BatchChunk *)(base + L.chunks);
    b->partials_d = (double2 *)(base + L.partials);
    b->sorted_d = (int32_t *)(base + L.sorted);
    b->pos_d = (int32_t *)(base + L.pos);
    b->counters_d = (uint32_t *)(base + L.counters);
    b->coef_d = (double2 *)(base + L.coef);
    hipStream_t s = (hipStream_t)stream;
    st = set_hip_error(hipMemcpyAsync(b->inst_d, inst.data(), sizeof(BatchInst) * count,
                                      hipMemcpyHostToDevice, s));
    if (!st) st = set_hip_error(hipMemcpyAsync(b->tile_prefix_d, prefix.data(),
                                                sizeof(int64_t) * (count + 1),
                                                hipMemcpyHostToDevice, s));
    if (!st) st = set_hip_error(hipMemcpyAsync(b->chunks_d, chunks.data(),
                                                sizeof(BatchChunk) * chunks.size(),
                                                hipMemcpyHostToDevice, s));
    if (!st) st = set_hip_error(hipMemcpyAsync(b->sorted_d, sorted.data(), sizeof(int32_t) * count,
                                                hipMemcpyHostToDevice, s));
    if (!st) st = set_hip_error(hipMemcpyAsync(b->pos_d, pos.data(), sizeof(int32_t) * count,
                                                hipMemcpyHostToDevice, s));
    // host staging vectors go out of scope: wait for the copies
    if (!st) st = set_hip_error(hipStreamSynchronize(s));
    if (st) {
        free(b->solo);
        free(b);
        return st;
    }
    *out = b;
    return MC_OK;
}

int mc_batch_destroy(mc_batch *b)
{
    if (b) free(b->solo);
    free(b);
    return MC_OK;
}

int64_t mc_batch_vector_length(const mc_batch *b) { return b ? b->total_len : (int64_t)MC_EINVAL; }

int mc_batch_apply_H(const mc_batch *b, const double *C_d, double *HC_d, mc_stream stream)
{
    if (!b || !C_d || !HC_d) return MC_EINVAL;
    if (overlaps(C_d, (size_t)b->total_len * 16, HC_d, (size_t)b->total_len * 16)) return MC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_batch_prep, dim3(4, b->count), dim3(256), 0, s, b->inst_d, b->counters_d);
    for (int k = 0; k < b->nsolo; ++k) {
        const SoloLaunch &L1 = b->solo[k];
        const int M = L1.M;
        const int64_t nblocks = (L1.tiles + 3) / 4;
#define MC_SOLO_LAUNCH(KIND)                                                                    \
    hipLaunchKernelGGL((k_batch_solo<MT, KIND>), dim3(nblocks), dim3(256), 0, s, L1.N,           \
                       bit_width(L1.N), L1.dim,                                                  \
                       L1.tiles, nblocks, L1.cap, L1.occ, L1.t1, L1.pmask, L1.t2_off, L1.t2,     \
                       (const double2 *)b->coef_d + L1.gp_off,                                   \
                       (const double2 *)b->coef_d + L1.hp_off,                                   \
                       (const double2 *)C_d + L1.vec_off, (double2 *)HC_d + L1.vec_off)
        switch (L1.kind) {
        case kPaperMap: MC_DISPATCH_M(M, if constexpr (MT > 0) MC_SOLO_LAUNCH(kPaperMap)); break;
        case kPaperChain: MC_DISPATCH_M(M, if constexpr (MT > 0) MC_SOLO_LAUNCH(kPaperChain)); break;
        case kSplitMap: MC_DISPATCH_M(M, if constexpr (MT > 0) MC_SOLO_LAUNCH(kSplitMap)); break;
        case kDirect: MC_DISPATCH_M(M, if constexpr (MT > 0) MC_SOLO_LAUNCH(kDirect)); break;
        default: MC_DISPATCH_M(M, if constexpr (MT > 0) MC_SOLO_LAUNCH(kSplitChain)); break;
        }
#undef MC_SOLO_LAUNCH
    }
    for (int gi = 0; gi < b->ngroups; ++gi) {
        const int M = b->group_M[gi];
#define MC_BATCH_LAUNCH(KIND)                                                                   \
    hipLaunchKernelGGL((k_batch_apply<MT, KIND>), dim3(b->group_blocks[gi]), dim3(256), 0, s,   \
                       b->inst_d, b->tile_prefix_d, b->group_first[gi], b->group_count[gi],     \
                       b->group_tiles[gi], b->group_blocks[gi], b->order, b->counters_d + gi,   \
                       (const double2 *)b->coef_d, (const double2 *)C_d, (double2 *)HC_d)
        switch (b->group_kind[gi]) {
        case kPaperMap: MC_DISPATCH_M(M, if constexpr (MT > 0) MC_BATCH_LAUNCH(kPaperMap)); break;
        case kPaperChain: MC_DISPATCH_M(M, if constexpr (MT > 0) MC_BATCH_LAUNCH(kPaperChain)); break;
        case kSplitMap: MC_DISPATCH_M(M, if constexpr (MT > 0) MC_BATCH_LAUNCH(kSplitMap)); break;
        case kDirect: MC_DISPATCH_M(M, if constexpr (MT > 0) MC_BATCH_LAUNCH(kDirect)); break;
        default: MC_DISPATCH_M(M, if constexpr (MT > 0) MC_BATCH_LAUNCH(kSplitChain)); break;
        }
#undef MC_BATCH_LAUNCH
    }
    return launch_status();
}

int mc_batch_dot(const mc_batch *b, const double *x_d, const double *y_d, double *out_d,
                 mc_stream stream)
{
    if (!b || !x_d || !y_d || !out_d) return MC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int64_t grid = b->nchunks < 4096 ? b->nchunks : 4096;
    hipLaunchKernelGGL(k_seg_dot_partial, dim3(grid), dim3(256), 0, s, b->chunks_d, b->nchunks,
                       (const double2 *)x_d, (const double2 *)y_d, b->partials_d);
    hipLaunchKernelGGL(k_seg_final, dim3((b->count + 255) / 256), dim3(256), 0, s, b->chunks_d,
                       b->nchunks, b->count, b->sorted_d, b->partials_d, (double2 *)out_d,
                       (double *)nullptr);
    return launch_status();
}

int mc_batch_lanczos_orth(const mc_batch *b, double *w_d, const double *v_d,
                          const double *vprev_d, const double *alpha_d, const double *beta_d,
                          mc_stream stream)
{
    if (!b || !w_d || !v_d || !alpha_d) return MC_EINVAL;
    const int64_t grid = b->nchunks < 8192 ? b->nchunks : 8192;
    hipLaunchKernelGGL(k_seg_orth, dim3(grid), dim3(256), 0, (hipStream_t)stream, b->chunks_d,
                       b->nchunks, b->sorted_d, (double2 *)w_d, (const double2 *)v_d,
                       (const double2 *)vprev_d, (const double2 *)alpha_d, beta_d);
    return launch_status();
}

int mc_batch_normalize(const mc_batch *b, const double *w_d, double *out_d, double *beta_d,
                       mc_stream stream)
{
    if (!b || !w_d || !out_d || !beta_d) return MC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int64_t grid = b->nchunks < 4096 ? b->nchunks : 4096;
    hipLaunchKernelGGL(k_seg_dot_partial, dim3(grid), dim3(256), 0, s, b->chunks_d, b->nchunks,
                       (const double2 *)w_d, (const double2 *)w_d, b->partials_d);
    hipLaunchKernelGGL(k_seg_final, dim3((b->count + 255) / 256), dim3(256), 0, s, b->chunks_d,
                       b->nchunks, b->count, b->sorted_d, b->partials_d, (double2 *)nullptr,
                       beta_d);
    const int64_t grid2 = b->nchunks < 8192 ? b->nchunks : 8192;
    hipLaunchKernelGGL(k_seg_scale, dim3(grid2), dim3(256), 0, s, b->chunks_d, b->nchunks,
                       b->sorted_d, (const double2 *)w_d, beta_d, (double2 *)out_d);
    return launch_status();
}

struct mc_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

int mc_batch_lanczos_graph(const mc_batch *b, int32_t steps, const double *v0_d, double *V_d,
                           double *w_d, double *alpha_d, double *beta_d, mc_stream stream,
                           mc_graph **out)
{
    if (!b || steps < 1 || !v0_d || !V_d || !w_d || !alpha_d || !beta_d || !out || !stream)
        return MC_EINVAL;
    *out = nullptr;
    const int64_t n = b->total_len;
    double *V[3] = {V_d, V_d + 2 * n, V_d + 4 * n};
    for (int i = 0; i < 3; ++i)
        if (overlaps(V[i], (size_t)n * 16, w_d, (size_t)n * 16)) return MC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    int st = set_hip_error(hipStreamIsCapturing(s, &cs));
    if (st) return st;
    if (cs != hipStreamCaptureStatusNone) return MC_EINVAL;
    st = set_hip_error(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    if (st) return st;
    // the recurrence; every call below only enqueues kernels
    int rec = mc_batch_normalize(b, v0_d, V[0], beta_d + (int64_t)steps * b->count, stream);
    for (int32_t j = 0; j < steps && rec == MC_OK; ++j) {
        double *cur = V[j % 3], *prev = V[(j + 2) % 3], *nxt = V[(j + 1) % 3];
        double *alpha_j = alpha_d + (int64_t)2 * j * b->count;
        rec = mc_batch_apply_H(b, cur, w_d, stream);
        if (rec == MC_OK) rec = mc_batch_dot(b, cur, w_d, alpha_j, stream);
        if (rec == MC_OK)
            rec = mc_batch_lanczos_orth(b, w_d, cur, j > 0 ? prev : nullptr, alpha_j,
                                        j > 0 ? beta_d + (int64_t)(j - 1) * b->count : nullptr,
                                        stream);
        if (rec == MC_OK) rec = mc_batch_normalize(b, w_d, nxt, beta_d + (int64_t)j * b->count, stream);
    }
    hipGraph_t graph = nullptr;
    st = set_hip_error(hipStreamEndCapture(s, &graph));
    if (rec != MC_OK || st != MC_OK) {
        if (graph) hipGraphDestroy(graph);
        return rec != MC_OK ? rec : st;
    }
    hipGraphExec_t exec = nullptr;
    st = set_hip_error(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    if (st) {
        hipGraphDestroy(graph);
        return st;
    }
    mc_graph *gr = (mc_graph *)malloc(sizeof(mc_graph));
    if (!gr) {
        hipGraphExecDestroy(exec);
        hipGraphDestroy(graph);
        return MC_ENOMEM;
    }
    gr->graph = graph;
    gr->exec = exec;
    *out = gr;
    return MC_OK;
}

int mc_graph_launch(const mc_graph *g, mc_stream stream)
{
    if (!g) return MC_EINVAL;
    return set_hip_error(hipGraphLaunch(g->exec, (hipStream_t)stream));
}

int mc_graph_destroy(mc_graph *g)
{
    if (!g) return MC_OK;
    int st = set_hip_error(hipGraphExecDestroy(g->exec));
    const int st2 = set_hip_error(hipGraphDestroy(g->graph));
    free(g);
    return st ? st : st2;
}

}  // extern "C"
