/*
 * mc.h -- C ABI of the MI355X (gfx950) library for bosonic
 * multiconfigurational operators: Fock-space hashing, single/double jump
 * maps, the many-body Hamiltonian apply H.C and the one/two-body reduced
 * density matrices, after Andriati & Gammal, arXiv:2005.13679.
 *
 * Operator conventions (paper, Sec. II):
 *   H = sum_{k,l} h_kl a+_k a_l + 1/2 sum_{k,s,q,l} g_ksql a+_k a+_s a_q a_l
 *   rho1_kl   = <Psi| a+_k a_l |Psi>                         (Eq. rho1)
 *   rho2_ksql = <Psi| a+_k a+_s a_q a_l |Psi>                (Eq. rho2)
 * Orbitals are 0..M-1, configurations are indexed 0..D-1 with
 * D = N_c(N, M) = C(N+M-1, N) (Eq. nc).  Index 0 is [N,0,...,0] and D-1 is
 * [0,...,0,N]: orbital M-1 is the most significant (Algorithms 1 and 2).
 *
 * General rules for every call:
 *   - Every function returns an int status (MC_OK = 0, negative on error)
 *     unless stated otherwise.  Nothing aborts, throws or prints.
 *   - The caller owns every buffer.  Pointers named *_d are device pointers
 *     (HIP device memory of the current device); all others are host.
 *   - Complex numbers are interleaved (re, im) doubles, i.e. complex128 /
 *     hipDoubleComplex.  Matrices are row-major: h[k*M + l],
 *     g[((k*M + s)*M + q)*M + l]; rho1 and rho2 use the same layouts.
 *   - Device work is enqueued asynchronously on `stream` (a hipStream_t;
 *     NULL = the null stream).  Argument errors are reported before anything
 *     is enqueued; launch errors return MC_EHIP with the HIP code available
 *     from mc_last_hip_error().  Faults inside kernels surface at the next
 *     synchronising call, as with any HIP work.
 *   - Sizes: 1 <= M <= MC_MAX_M, 1 <= N <= MC_MAX_N, and every call that
 *     uses jump tables needs D < 2^31 (int32 table entries).
 */
#ifndef MC_H
#define MC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MC_OK       0
#define MC_EINVAL  -1   /* bad argument: N, M, null pointer, occupation sum != N, aliasing */
#define MC_ERANGE  -2   /* index outside [0, D), dimension or table size overflow */
#define MC_ENOMEM  -3   /* a caller buffer or workspace is too small */
#define MC_EHIP    -4   /* a HIP call failed; see mc_last_hip_error() */

#define MC_MAX_M    32
#define MC_MAX_N    65535
#define MC_TILE     64  /* rows per tile: one wavefront lane per row */

typedef void *mc_stream;   /* hipStream_t */

/* Human-readable text for a status code (static storage). */
const char *mc_strerror(int status);

/* The last hipError_t value returned to the library on the calling thread
 * (0 if none).  Reading it does not clear it. */
int mc_last_hip_error(void);

/* ------------------------------------------------------------------------ */
/* Combinatorics (host only, no device work)                                */
/* ------------------------------------------------------------------------ */

/* Dimension N_c(N, M) = (N+M-1)! / (N! (M-1)!)  (Eq. nc).
 * Returns D >= 1, or MC_EINVAL for N < 0 or M < 1, or MC_ERANGE if D does
 * not fit in int64. */
int64_t mc_dim(int32_t N, int32_t M);

/* Configuration -> index: the perfect hash of Eq. (TotalCost) / Algorithm 1.
 * occ[M] holds the occupations (each >= 0, sum == N).  Writes *index.
 * MC_EINVAL on a bad occupation vector or null pointer. */
int mc_hash(int32_t N, int32_t M, const int32_t *occ, int64_t *index);

/* Index -> configuration (Algorithm 2).  Writes occ[M].
 * MC_ERANGE if index is outside [0, D). */
int mc_unhash(int32_t N, int32_t M, int64_t index, int32_t *occ);

/* ------------------------------------------------------------------------ */
/* Tables: the hashing table and the single/double jump maps (Secs. III-IV) */
/* ------------------------------------------------------------------------ */
/*
 * All tables are stored in 64-row tiles: tile t covers rows 64t .. 64t+63,
 * row r of the tile sits in wavefront lane r, and rows >= D are padding.
 *
 *   binom   int64 [N+3][M+1]        binom[x][m] = C(x+m, m)
 *   occ     [tiles][M][64]          occupation n_m of row 64t+lane; uint8 if
 *                                   N <= 255 else uint16 (the "hashing table")
 *   t1      int32 [tiles][M][M][64] single-jump map: index after moving one
 *                                   particle k -> l, -1 if n_k = 0; k = l
 *                                   gives the row itself (n_k >= 1)
 *   pmask   uint64 [tiles][W]       bit p set if any row of the tile has
 *                                   removal pair p valid; W = ceil(P/64),
 *                                   P = M(M+1)/2 pairs (k <= s) in
 *                                   lexicographic order
 *   t2_off  int64 [tiles+1]         start of each tile in t2 (entries)
 *   t2      int32 [t2_off[tiles]]   double-jump map.  For each removal pair
 *                                   p with its pmask bit set, in increasing
 *                                   p, a block of M*M*64 entries:
 *                                   entry (q*M + l)*64 + lane is the index
 *                                   after removing one particle from k and
 *                                   one from s and adding one to q and one
 *                                   to l, or -1 if the pair is not valid
 *                                   for that row (k = s needs n_k >= 2,
 *                                   k < s needs n_k >= 1 and n_s >= 1).
 *
 * The double-jump content is exactly the paper's variable-length rows
 * (Sec. IV, Fig. jump_illustration): per row, a stride of M^2 entries per
 * valid removal pair in lexicographic order, slot q*M + l.  Only the memory
 * order differs: tiles are stored slot-major so that 64 consecutive rows
 * read 64 consecutive entries.
 *
 * Reduced form (t->form == MC_FORM_REDUCED).  A slot whose creation pair
 * {q, l} shares an orbital with the removal pair {k, s} leads back to the row
 * itself or to a single jump (the coincident-index cases of the appendix on
 * matrix elements), and slots (q, l) and (l, q) lead to the same
 * configuration.  The reduced map keeps one entry per true double jump: the
 * block of pair (k, s) holds nd(k, s) * 64 entries, slot r being the r-th
 * creation pair (q, l), q <= l, q and l both outside {k, s}, in
 * lexicographic order; nd = M(M-1)/2 for k = s and (M-1)(M-2)/2 for k < s
 * (110 entries per full row at M = 5 instead of 375).  Offsets, pair mask
 * and padding follow the same rules with these block sizes.
 */
#define MC_FORM_PAPER 0     /* double-jump map as in the paper (M^2 slots per pair) */
#define MC_FORM_REDUCED 1   /* true double jumps only (see above) */
typedef struct mc_table_sizes {
    int64_t dim;            /* D */
    int64_t tiles;          /* ceil(D / 64) */
    int32_t occ_bytes;      /* bytes per occupation: 1 or 2 */
    int32_t pair_words;     /* W */
    int64_t binom_bytes;
    int64_t occ_bytes_total;
    int64_t t1_bytes;
    int64_t pmask_bytes;
    int64_t t2_off_bytes;
    int64_t t2_compact_entries; /* entries of the paper's packed rows:
                                   M^2 * M(M+1)/2 * N_c(N-2, M) */
    int64_t t2r_compact_entries; /* entries of the reduced rows:
                                    [M * M(M-1)/2 + M(M-1)/2 * (M-1)(M-2)/2]
                                    * N_c(N-2, M) */
} mc_table_sizes;

/* Sizes of every table for (N, M).  Host only.  MC_ERANGE if D >= 2^31. */
int mc_tables_size(int32_t N, int32_t M, mc_table_sizes *out);

/* Device bytes the tables of (N, M) take in `form`: binomials, occupations,
 * single-jump map, pair mask and offsets, plus (with_double_jumps != 0) the
 * tiled double-jump map at its largest, i.e. with a block for every removal
 * pair in every tile (a built map is at most this; the exact size is
 * t2_required after mc_build_jump_tables).  Host only; errors as
 * mc_tables_size, MC_EINVAL for an unknown form. */
int mc_tables_bytes(int32_t N, int32_t M, int32_t form, int32_t with_double_jumps,
                    int64_t *bytes);

/* HBM budget for the double-jump maps of many instances (a batch): keep[i]
 * = 1 for the instances that get a map, 0 for those that chain single jumps
 * instead.  Maps (sized as in mc_tables_bytes) are admitted smallest first,
 * ties by position, while their total stays within budget_bytes, so the most
 * instances are served.  N[count], M[count], keep[count] are host arrays.
 * Host only; MC_EINVAL / MC_ERANGE for a bad instance. */
int mc_choose_double_jumps(int32_t count, const int32_t *N, const int32_t *M, int32_t form,
                           double budget_bytes, int32_t *keep);

typedef struct mc_tables {
    int32_t N, M;
    int64_t dim, tiles;
    int64_t *binom_d;
    void *occ_d;
    int32_t *t1_d;
    uint64_t *pmask_d;
    int64_t *t2_off_d;
    int32_t *t2_d;           /* may be NULL until mc_build_double_jumps */
    int64_t t2_entries;      /* capacity of t2_d, in entries */
    int64_t t2_required;     /* set by mc_build_jump_tables */
    int32_t form;            /* MC_FORM_PAPER or MC_FORM_REDUCED; set before
                                mc_build_jump_tables (it fixes t2_off) */
    int32_t reserved;
} mc_tables;

/* Builds binom, occ, t1, pmask and t2_off into the caller's buffers (sizes
 * from mc_tables_size; t->N, t->M must match; t->form picks the block sizes
 * of t2_off).  Synchronises `stream` once at the end to read t2_off[tiles]
 * into t->t2_required (entries the double jump map needs).  MC_EINVAL on a
 * missing buffer, mismatched N/M or an unknown form. */
int mc_build_jump_tables(int32_t N, int32_t M, mc_tables *t, mc_stream stream);

/* Fills t->t2_d in the tables' form.  Needs a completed mc_build_jump_tables
 * on the same tables (same form) and t->t2_entries >= t->t2_required (else
 * MC_ENOMEM). */
int mc_build_double_jumps(int32_t N, int32_t M, const mc_tables *t, mc_stream stream);

/* Device-side hash / unhash of many configurations, row-major int32
 * occupations occ_d[count][M].  The binomial table comes from built tables
 * (only t->binom_d is read).  Invalid rows produce -1 (hash) or a row of -1
 * (unhash); nothing faults. */
int mc_hash_batch(int32_t N, int32_t M, const mc_tables *t, const int32_t *occ_d,
                  int64_t *index_d, int64_t count, mc_stream stream);
int mc_unhash_batch(int32_t N, int32_t M, const mc_tables *t, const int64_t *index_d,
                    int32_t *occ_d, int64_t count, mc_stream stream);

/* Reads the double-jump map entry for (row, k, s, q, l) of each query
 * (queries_d[count][5] int64: row, k, s, q, l with any k, s order) into
 * out_d[count]; -1 where the removal is not possible.  A test and debugging
 * accessor for the tiled layout; paper form only (MC_EINVAL otherwise). */
int mc_t2_lookup(int32_t N, int32_t M, const mc_tables *t, const int64_t *queries_d,
                 int32_t *out_d, int64_t count, mc_stream stream);

/* ------------------------------------------------------------------------ */
/* Operators                                                                */
/* ------------------------------------------------------------------------ */

#define MC_OP_APPLY 1
#define MC_OP_RHO1  2
#define MC_OP_RHO2  3
#define MC_OP_DOT   4
#define MC_OP_RHO1_DIRECT 5
#define MC_OP_RHO2_DIRECT 6

/* Bytes of device workspace `op` needs for (N, M) (0 is possible). */
int mc_workspace_size(int32_t N, int32_t M, int32_t op, size_t *bytes);

/* HC_d = H . C_d  (Eq. Haction), matrix-free through the jump maps:
 *   (H C)_g = sum_k h_kk n_k C_g
 *           + sum_{k != l, n_k >= 1} h_kl sqrt(n_k (n_l+1)) C[t1[g][k][l]]
 *           + 1/2 sum_{valid pairs k<=s} A_ks sum_{q,l} G'_{ks,ql} B_ql C[t2 slot]
 * with G'_{ks,ql} = g_ksql + g_skql (k < s), g_kkql (k = s),
 * A_ks = sqrt(n_k n_s) or sqrt(n_k(n_k-1)), and B_ql the creation amplitudes
 * on m = n - e_k - e_s (sqrt((m_q+1)(m_l+1)), or sqrt((m_q+1)(m_q+2)) if
 * q = l).  If the tables were built without the double-jump map
 * (t->t2_d == NULL), each double-jump target is found as two chained single
 * jumps, T1[T1[g][k][q]][s][l] (M <= 8), and no double-jump table is read.
 *
 * Tables in the reduced form (M <= 8) evaluate the same sum case by case:
 * slots with {q,l} = {k,s} add to the row's own coefficient, slots sharing
 * one orbital add to the single-jump coefficients, and only the true double
 * jumps are gathered (reduced map, or chained single jumps without it):
 *   (H C)_g = [sum_k n_k (h_kk - I_kk) + sum_{k<=s} n_k n_s I_ks] C_g
 *           + sum_{a != b} sqrt(n_a (n_b+1)) [h_ab - S_aba + sum_c n_c S_abc]
 *                                                       C[t1[g][a][b]]
 *           + sum_{valid k<=s} A_ks sum_{q<=l outside {k,s}} B_ql(n) R_ks,ql
 *                                                       C[reduced slot]
 * with g' = G'/2 the staged pair coefficients, I_ks = g'_{ks,ks} + g'_{ks,sk}
 * (k < s) or g'_{kk,kk}; S_abc = g'_{ac,cb} + g'_{ac,bc} (c != b) or
 * g'_{ab,bb}, taken over the unordered pair {a, c}; R_ks,ql = g'_{ks,ql} +
 * g'_{ks,lq} (q < l) or g'_{ks,qq}.  Sums agree with the paper form up to
 * rounding order.
 * h_d [M*M], g_d [M^4], C_d and HC_d [D] complex128 on the device;
 * HC_d must not overlap C_d (MC_EINVAL).  ws_d: mc_workspace_size(APPLY);
 * the call stages h and G' there, so concurrent calls need separate ws.
 * No symmetry of h or g is assumed. */
/* Table reads of the apply through a double-jump map (host query, no
 * device work).  Within a run of rows (consecutive indices that differ by one
 * particle moved between orbitals 0 and 1, Eq. TotalCost) a jump's target is
 * the row's index plus a constant of the run and of the jump's class (the
 * jumps that change the prefix sums S_1 .. S_{M-2} alike), so on a tile where
 * every removal pair occurs (2 <= M <= 6) the kernel reads from the tables
 * only one jump per class and derives the others' targets; slots with one
 * target share one coefficient.  form: MC_FORM_PAPER (single jumps and the
 * M*M slots of every removal pair) or MC_FORM_REDUCED (single jumps and the
 * true double jumps).  *slots: jump slots per row; *table_columns: those
 * read from the tables per such tile.  Larger M: every slot is read
 * (*table_columns = *slots).  MC_EINVAL for M outside 1..8, an unknown form
 * or NULL outputs. */
int mc_apply_stream_columns(int32_t M, int32_t form, int32_t *slots, int32_t *table_columns);

int mc_apply_H(int32_t N, int32_t M, const double *h_d, const double *g_d,
               const mc_tables *t, const double *C_d, double *HC_d,
               void *ws_d, size_t ws_bytes, mc_stream stream);

/* HC_d = H^dagger . C_d, the same apply with h -> h^dagger
 * (conj(h_lk)) and g -> g^dagger (g^dagger_ksql = conj(g_lqsk)).  Equals
 * mc_apply_H when H is Hermitian; needed for gradients of E = <C|H C> with
 * non-Hermitian inputs.  Same arguments and errors as mc_apply_H. */
int mc_apply_H_adjoint(int32_t N, int32_t M, const double *h_d, const double *g_d,
                       const mc_tables *t, const double *C_d, double *HC_d,
                       void *ws_d, size_t ws_bytes, mc_stream stream);

/* HC_d = H . C_d in the case-split form of mc_apply_H, for interactions
 * most of whose coefficients vanish (e.g. momentum conservation of the
 * plane-wave g of the Lieb-Liniger model, Sec. VI: 44 of 462 true double
 * jumps per row survive at M = 7, and no single-jump term).  After staging,
 * one kernel lists the single jumps and reduced slots whose constants are not
 * all zero; the apply gathers only those.  Needs reduced-form tables (with or
 * without the map) and M <= 8, else MC_EINVAL; other arguments as mc_apply_H.
 * Results equal mc_apply_H's up to rounding order for any g. */
int mc_apply_H_sparse(int32_t N, int32_t M, const double *h_d, const double *g_d,
                      const mc_tables *t, const double *C_d, double *HC_d,
                      void *ws_d, size_t ws_bytes, mc_stream stream);

/* HC_d = H . C_d with no table: the case-split sum of mc_apply_H, with each
 * row's occupations and each jump target computed from the row's index in
 * closed form instead of read from the hashing table and the jump maps.
 * Summing Eq. TotalCost over the particles of each orbital gives
 *   g = D - 1 - sum_{m=0}^{M-2} C(S_m + m, m + 1),  S_m = n_0 + ... + n_m,
 * so the occupations follow from g greedily and a jump, which shifts a few
 * S_m by at most 2, changes g by a sum of at most M-1 precomputed per-row
 * differences (the O(M) index delta; Sec. III, IV).  Needs no mc_tables:
 * device memory is C_d, HC_d and the workspace only, which lifts the table
 * memory limit on N.  1 <= M <= 8 and D < 2^31 (else MC_EINVAL / MC_ERANGE),
 * (N+3)*8 <= 65536 for M >= 5 (an LDS table of square roots; M <= 4 keeps
 * them in registers); ws_d: mc_workspace_size(APPLY) bytes (staged constants,
 * so concurrent calls need separate ws); HC_d must not overlap C_d.  The
 * terms and their order are those of mc_apply_H on reduced-form tables, so
 * the results agree with it up to the sign of zero. */
int mc_apply_H_direct(int32_t N, int32_t M, const double *h_d, const double *g_d,
                      const double *C_d, double *HC_d, void *ws_d, size_t ws_bytes,
                      mc_stream stream);

/* mc_apply_H_direct without a workspace argument, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the call itself allocates nothing.  The staged constants
 * go to a device array owned by the library, MC_NOALLOC_SCRATCH_BYTES bytes,
 * one per GPU, held until the process ends; its address is looked up once per
 * device, on the first call with that device current.  Every call on a GPU
 * shares that GPU's array and the last call's constants stay in it: calls on
 * one stream are ordered, calls that overlap on one GPU (other streams, other
 * host threads) race.  MC_ENOMEM if the constants of (N, M) exceed the array
 * (never for M <= 8); other arguments, limits and errors as
 * mc_apply_H_direct, whose kernels it runs. */
#define MC_NOALLOC_SCRATCH_BYTES 65536
int mc_apply_H_direct_noalloc(int32_t N, int32_t M, const double *h_d, const double *g_d,
                              const double *C_d, double *HC_d, mc_stream stream);

/* HC_d = H^dagger . C_d with no table (h -> h^dagger, g_ksql -> conj(g_lqsk)),
 * the table-free counterpart of mc_apply_H_adjoint; arguments, limits and
 * errors as mc_apply_H_direct. */
int mc_apply_H_direct_adjoint(int32_t N, int32_t M, const double *h_d, const double *g_d,
                              const double *C_d, double *HC_d, void *ws_d, size_t ws_bytes,
                              mc_stream stream);

/* flag_d[0] (int32, device) = 1 if h_kl == conj(h_lk) for all k, l and
 * g_ksql == conj(g_lqsk) for all k, s, q, l (exact comparisons), else 0.  In
 * the first case H^dagger = H (Sec. II) and mc_apply_H_adjoint equals
 * mc_apply_H; the energy gradient uses this to skip the adjoint apply.  The
 * test is sufficient, not necessary: a g that is Hermitian only after the
 * k <-> s, q <-> l symmetrisation gives 0.  One small kernel on `stream`. */
int mc_is_hermitian(int32_t M, const double *h_d, const double *g_d, int32_t *flag_d,
                    mc_stream stream);

/* rho1_d [M*M] = <a+_k a_l> (Eq. rho1) through the single-jump map.
 * Deterministic fixed-order reduction in ws_d (mc_workspace_size(RHO1)). */
int mc_rho1(int32_t N, int32_t M, const mc_tables *t, const double *C_d,
            double *rho1_d, void *ws_d, size_t ws_bytes, mc_stream stream);

/* rho2_d [M^4] = <a+_k a+_s a_q a_l> (Eq. rho2) through the double-jump map,
 * deterministic fixed-order reduction in ws_d (mc_workspace_size(RHO2)).
 * Needs a double-jump map (either form; in the reduced form the slots that
 * share an orbital with the removal pair read the row itself or the
 * single-jump map, App. B's coincident-index cases), M <= 8. */
int mc_rho2(int32_t N, int32_t M, const mc_tables *t, const double *C_d,
            double *rho2_d, void *ws_d, size_t ws_bytes, mc_stream stream);

/* rho1_d [M*M] (Eq. rho1) and rho2_d [M^4] (Eq. rho2) with no table, as
 * Gram matrices over the configurations m of N-1 and N-2 particles:
 *   rho_kl   = sum_m conj(X1_m[k]) X1_m[l],   X1_m[l] = sqrt(m_l+1) C[m + e_l],
 *   rho_ksql = sum_m conj(X2_m[ks]) X2_m[ql],
 *   X2_m[ql] = sqrt((m_q+1)(m_l+1+[q=l])) C[m + e_q + e_l]
 * (the annihilators of Eqs. rho1, rho2 applied to the ket; ladder
 * amplitudes of Sec. II).  The index of m + e_q + e_l follows from m's
 * prefix sums in closed form, as in mc_apply_H_direct.  Only the upper
 * triangle over unordered pairs is accumulated; the rest follows from
 * rho_ksql = rho_skql = rho_kslq = conj(rho_qlks) (and rho_lk = conj(rho_kl)),
 * diagonal entries are real.  N < 1 (rho1) or N < 2 (rho2) gives zeros.
 * 1 <= M <= 8 (MC_EINVAL), D < 2^31 (MC_ERANGE).  ws_d: at least
 * mc_workspace_size(MC_OP_RHO1_DIRECT / MC_OP_RHO2_DIRECT) bytes (per-
 * wavefront partials and their fixed-order sum: bitwise reproducible), else
 * MC_ENOMEM.  Results equal mc_rho1 / mc_rho2 up to rounding order. */
int mc_rho1_direct(int32_t N, int32_t M, const double *C_d, double *rho1_d, void *ws_d,
                   size_t ws_bytes, mc_stream stream);
int mc_rho2_direct(int32_t N, int32_t M, const double *C_d, double *rho2_d, void *ws_d,
                   size_t ws_bytes, mc_stream stream);

/* out_d[1] complex = sum_i conj(x_i) y_i over n elements, fixed-order
 * reduction in ws_d (mc_workspace_size(DOT) for n = D of (N, M), or any
 * ws of at least 16 * MC_DOT_BLOCKS + 16 bytes). */
#define MC_DOT_BLOCKS 1024
int mc_zdotc(int64_t n, const double *x_d, const double *y_d, double *out_d,
             void *ws_d, size_t ws_bytes, mc_stream stream);

/* out_d[i] = scale * (op(a) op(x_i) + op(b) op(y_i)) for i < n, complex128,
 * with device scalars a_d, b_d (NULL = 1) and op = complex conjugation where
 * the matching MC_CONJ_* bit of `flags` is set; y_d = NULL drops the second
 * term.  out_d may alias x_d or y_d element-wise.  Used for the gradient
 * combinations of the energy functional (no host arithmetic in the path). */
#define MC_CONJ_A 1u
#define MC_CONJ_X 2u
#define MC_CONJ_B 4u
#define MC_CONJ_Y 8u
int mc_zaxpby(int64_t n, const double *a_d, const double *x_d, const double *b_d,
              const double *y_d, double scale, uint32_t flags, double *out_d, mc_stream stream);

/* ------------------------------------------------------------------------ */
/* Batches of instances of uneven size                                      */
/* ------------------------------------------------------------------------ */
/*
 * A batch applies H_i to C_i for many instances i = (N_i, M_i, h_i, g_i) at
 * once.  A batch vector is the concatenation of the instances' coefficient
 * vectors in the order the caller lists them (instance i at offset
 * sum_{j<i} D_j, total mc_batch_vector_length()).  Instances are grouped by
 * orbital count and by how their tiles run (paper or reduced form, with or
 * without a double-jump map); each group runs as one persistent kernel whose
 * wavefronts walk the group's (instance, 64-row tile) work list.  An
 * instance whose tables hold a double-jump map uses it; one built without it
 * (t2_d == NULL) chains two single jumps; reduced-form tables run the
 * case-split sum of mc_apply_H.  Limits per instance: M <= 8, N <= 255,
 * D < 2^28.
 *
 * Every batch call only enqueues kernels on `stream` (no host
 * synchronisation, no memset), so sequences of calls can be captured into a
 * HIP graph and replayed.  A batch's plan holds staged coefficients and work
 * counters: applies of one batch that overlap in time (other streams) race;
 * calls on one stream are ordered.
 */
typedef struct mc_batch_item {
    const mc_tables *tables;     /* host pointer to built tables of the instance, or to a
                                    descriptor with N, M, dim, tiles set and every buffer
                                    pointer NULL: the instance then runs table-free (the
                                    evaluation of mc_apply_H_direct) */
    const double *h_d, *g_d;     /* h [M*M], g [M^4] complex128, device; read at each apply */
} mc_batch_item;

typedef struct mc_batch_schedule {
    int32_t blocks_per_cu;   /* persistent grid per group: blocks_per_cu x CUs blocks of
                                256 threads (0 = 2) */
    int32_t order;           /* 0: wavefront w takes work items w, w+W, ...; 1: each
                                wavefront takes a contiguous range of items; 2: each
                                XCD takes a contiguous share of the items (in
                                proportion to its blocks) and its wavefronts
                                interleave within it; 3: wavefronts take 8 items at
                                a time from a per-group counter in the plan (zeroed
                                by a kernel at the start of each apply) */
    int32_t solo_tiles;      /* > 0: an instance of at least this many 64-row tiles
                                gets a launch of its own (one wavefront per tile, like
                                mc_apply_H) instead of joining its group's persistent
                                kernel; 0: every instance joins its group */
    int32_t reserved;
} mc_batch_schedule;

typedef struct mc_batch mc_batch;   /* opaque host handle */

/* Bytes of the device plan buffer mc_batch_create needs. */
int mc_batch_plan_size(int32_t count, const mc_batch_item *items, size_t *bytes);

/* Builds the plan into plan_d (caller-owned device memory, plan_bytes >=
 * mc_batch_plan_size) and returns a host handle in *out (free with
 * mc_batch_destroy).  Synchronises `stream` once (plan upload).  The tables
 * and h/g buffers must outlive the handle. */
int mc_batch_create(int32_t count, const mc_batch_item *items, const mc_batch_schedule *sched,
                    void *plan_d, size_t plan_bytes, mc_stream stream, mc_batch **out);
int mc_batch_destroy(mc_batch *b);
int64_t mc_batch_vector_length(const mc_batch *b);

/* HC_d = H_i C_d per instance segment (batch vectors, no overlap). */
int mc_batch_apply_H(const mc_batch *b, const double *C_d, double *HC_d, mc_stream stream);

/* out_d[i] = <x_i | y_i> (complex128 per instance, caller order), fixed-order
 * reductions. */
int mc_batch_dot(const mc_batch *b, const double *x_d, const double *y_d, double *out_d,
                 mc_stream stream);

/* Per instance: w_i -= Re(alpha_d[i]) v_i + beta_d[i] vprev_i (alpha complex128,
 * beta double; vprev_d or beta_d NULL drops the second term). */
int mc_batch_lanczos_orth(const mc_batch *b, double *w_d, const double *v_d,
                          const double *vprev_d, const double *alpha_d, const double *beta_d,
                          mc_stream stream);

/* Per instance: beta_d[i] = ||w_i||, out_i = w_i / beta_d[i] (0 if beta = 0). */
int mc_batch_normalize(const mc_batch *b, const double *w_d, double *out_d, double *beta_d,
                       mc_stream stream);

/* A captured sequence of batch calls, replayed as one HIP graph. */
typedef struct mc_graph mc_graph;

/* Captures `steps` three-term Lanczos steps (no reorthogonalisation; the
 * recurrence of Sec. VI) of every instance of batch b into one HIP graph:
 *   normalize(v0) -> V[0], beta row `steps`;
 *   step j: apply(V[j%3]) -> w; dot(V[j%3], w) -> alpha row j;
 *           orth(w, V[j%3], V[(j-1)%3], alpha row j, beta row j-1);
 *           normalize(w) -> V[(j+1)%3], beta row j.
 * All device buffers: v0_d (batch vector, read at every launch), V_d (three
 * batch vectors back to back), w_d (batch vector, no overlap with V_d),
 * alpha_d complex128 [steps][count], beta_d double [steps+1][count]; each
 * row in the caller's instance order.  `stream` must be a non-null stream
 * that is not capturing; the capture (thread-local mode) enqueues nothing,
 * so nothing runs until mc_graph_launch.  Free with mc_graph_destroy; the
 * batch and every buffer must outlive the graph.  MC_EINVAL on bad
 * arguments, MC_EHIP if capture or instantiation fails. */
int mc_batch_lanczos_graph(const mc_batch *b, int32_t steps, const double *v0_d, double *V_d,
                           double *w_d, double *alpha_d, double *beta_d, mc_stream stream,
                           mc_graph **out);
/* Enqueues one replay of the graph on `stream`. */
int mc_graph_launch(const mc_graph *g, mc_stream stream);
int mc_graph_destroy(mc_graph *g);

/* ------------------------------------------------------------------------ */
/* Lanczos building blocks (Sec. VI: Lanczos tridiagonalisation with full   */
/* reorthogonalisation).  Scalars stay on the device.                        */
/* ------------------------------------------------------------------------ */

/* c_d[k] = sum_i conj(V_d[k*ldv + i]) w_d[i] for k < K (complex128), each a
 * fixed-order reduction.  ws_d: K * 64 * 16 bytes. */
int mc_zgemv_c(int32_t K, int64_t n, const double *V_d, int64_t ldv, const double *w_d,
               double *c_d, void *ws_d, size_t ws_bytes, mc_stream stream);

/* w_d[i] -= sum_{k<K} V_d[k*ldv + i] c_d[k] (complex128), k in order. */
int mc_zgemv_sub(int32_t K, int64_t n, const double *V_d, int64_t ldv, const double *c_d,
                 double *w_d, mc_stream stream);

/* beta = ||w_d|| (fixed-order reduction), out_d = w_d / beta (0 if beta = 0);
 * beta is written to beta_d[0] (double, may be NULL).  out_d may equal w_d.
 * ws_d: (MC_DOT_BLOCKS + 2) * 16 bytes. */
int mc_normalize(int64_t n, const double *w_d, double *out_d, double *beta_d, void *ws_d,
                 size_t ws_bytes, mc_stream stream);

/* Three-term Lanczos step without reorthogonalisation:
 * w_d -= Re(alpha_d[0]) v_d + beta_prev_d[0] vprev_d  (complex128 vectors,
 * alpha complex128 and beta double on the device; vprev_d or beta_prev_d
 * NULL drops the second term). */
int mc_lanczos_orth(int64_t n, double *w_d, const double *v_d, const double *vprev_d,
                    const double *alpha_d, const double *beta_prev_d, mc_stream stream);

/* out_d[i] = sum_{k<K} V_d[k*ldv + i] c_d[k] (complex128), k in order; the
 * Krylov combination of a Short Iterative Lanczos step.  out_d must not
 * overlap V_d (MC_EINVAL).  K >= 1. */
int mc_zgemv_n(int32_t K, int64_t n, const double *V_d, int64_t ldv, const double *c_d,
               double *out_d, mc_stream stream);

/* y = exp(-i T dt) e_0 (y[2K], interleaved complex, host) for the real
 * symmetric tridiagonal T with diagonal alpha[K] and off-diagonal beta[K-1]
 * (host arrays), through the eigen-decomposition of T by cyclic Jacobi
 * rotations: the small-matrix step of the Short Iterative Lanczos integrator
 * that Sec. II names for time-dependent problems (C(t+dt) ~ |C| V_K y).
 * 1 <= K <= 512, else MC_EINVAL.  Host only. */
int mc_tridiag_expv(int32_t K, const double *alpha, const double *beta, double dt, double *y);

/* Coefficients of a Short Iterative Lanczos step (Sec. II) after K Lanczos
 * steps of (H, C/|C|) with coefficients alpha[K], beta[K-1] and the norm
 * beta_next left after step K: coef[2K] (interleaved complex, host) =
 * norm_c * exp(-i T_K dt) e_0, so that C(t+dt) ~ sum_j coef_j v_j
 * (mc_zgemv_n); *err = norm_c * beta_next * |y_{K-1}|, the weight the next
 * Krylov vector would receive (the step's error estimate); *invariant = 1
 * and *err = 0 when beta_next < 1e-14 max(1, |alpha[K-1]|) (the Krylov space
 * is invariant and the step exact), else 0.  Host only; MC_EINVAL as
 * mc_tridiag_expv or for a null output. */
int mc_sil_coefficients(int32_t K, const double *alpha, const double *beta, double beta_next,
                        double norm_c, double dt, double *coef, double *err, int32_t *invariant);

/* Lowest eigenvalue of the real symmetric tridiagonal matrix with diagonal
 * alpha[K] and off-diagonal beta[K-1] (host arrays), by Sturm-sequence
 * bisection.  Host only. */
int mc_tridiag_lowest(int32_t K, const double *alpha, const double *beta, double *e0);

#ifdef __cplusplus
}
#endif

#endif /* MC_H */
