// Density matrices through the jump maps (Eqs. rho1, rho2; Sec. IV): the Gram
// kernels of mc_gram.h with each intermediate configuration m reached from
// the row m + L e_0 of the hashing table, its single jumps out of orbital 0
// and the (0, 0) block of the double-jump map (or two chained single jumps
// when the tables have no map).
#include "mc_gram.h"

namespace mc {
namespace {

template <int MT, int L, typename OT, int KIND, bool BIG>
int map_launch(const mc_tables *t, const GramShape &gs, const double *C_d, double *out_d,
               void *ws_d, hipStream_t s)
{
    MapSource<MT, L, OT, KIND, BIG> src;
    src.D = t->dim;
    src.cap = t->t2_d ? t->t2_entries : 0;
    src.occ = (const OT *)t->occ_d;
    src.t1 = t->t1_d;
    src.pmask = t->pmask_d;
    src.t2_off = t->t2_off_d;
    src.t2 = t->t2_d;
    return gram_launch<MT, L, BIG>(src, t->dim, gs, C_d, out_d, ws_d, s);
}

// KIND from the tables: 0 without a double-jump map, 1 paper form, 2 reduced
template <int MT, int L, typename OT, bool BIG>
int map_kind(const mc_tables *t, const GramShape &gs, const double *C_d, double *out_d,
             void *ws_d, hipStream_t s)
{
    if (L == 1 || !t->t2_d) return map_launch<MT, L, OT, 0, BIG>(t, gs, C_d, out_d, ws_d, s);
    if (t->form == MC_FORM_REDUCED) return map_launch<MT, L, OT, 2, BIG>(t, gs, C_d, out_d, ws_d, s);
    return map_launch<MT, L, OT, 1, BIG>(t, gs, C_d, out_d, ws_d, s);
}

template <int MT, int L>
int map_rho_t(const mc_tables *t, const GramShape &gs, const double *C_d, double *out_d,
              void *ws_d, hipStream_t s)
{
    const bool big = t->dim * 16 > (int64_t)0xFFFFFFFFu;
    if (occ_width(t->N) == 1) {
        if (big) return map_kind<MT, L, uint8_t, true>(t, gs, C_d, out_d, ws_d, s);
        return map_kind<MT, L, uint8_t, false>(t, gs, C_d, out_d, ws_d, s);
    }
    // more than 255 particles fit below 2^31 rows only for M <= 5
    if constexpr (MT <= 5) {
        if (big) return map_kind<MT, L, uint16_t, true>(t, gs, C_d, out_d, ws_d, s);
        return map_kind<MT, L, uint16_t, false>(t, gs, C_d, out_d, ws_d, s);
    }
    return MC_EINVAL;
}

int map_rho(int L, int32_t N, int32_t M, const mc_tables *t, const double *C_d, double *out_d,
            void *ws_d, size_t ws_bytes, mc_stream stream)
{
    int st = check_nm(N, M);
    if (st) return st;
    st = check_tables(N, M, t, false);
    if (st) return st;
    if (t->t2_d && t->t2_entries < t->t2_required) return MC_ENOMEM;
    if (!C_d || !out_d) return MC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (N < L) return gram_zero(M, L, out_d, s);
    GramShape gs;
    st = gram_shape(M, L, t->tiles, &gs);
    if (st) return st;
    if (!ws_d) return MC_EINVAL;
    if (ws_bytes < gs.ws) return MC_ENOMEM;
    MC_DISPATCH_M(M, if constexpr (MT > 0 && MT <= 8) {
        st = L == 1 ? (map_rho_t<MT, 1>)(t, gs, C_d, out_d, ws_d, s)
                    : (map_rho_t<MT, 2>)(t, gs, C_d, out_d, ws_d, s);
    });
    return st;
}

}  // namespace

size_t gram_table_workspace(int32_t N, int32_t M, int L)
{
    if (M > 8 || N < L) return 16;
    const int64_t D = dim_checked(N, M);
    if (D < 0) return 0;
    GramShape gs;
    if (gram_shape(M, L, (D + kTile - 1) / kTile, &gs)) return 0;
    return gs.ws;
}

}  // namespace mc

using namespace mc;

extern "C" {

int mc_rho1(int32_t N, int32_t M, const mc_tables *t, const double *C_d, double *rho1_d,
            void *ws_d, size_t ws_bytes, mc_stream stream)
{
    if (M > 8) return rho1_generic(N, M, t, C_d, rho1_d, ws_d, ws_bytes, stream);
    return map_rho(1, N, M, t, C_d, rho1_d, ws_d, ws_bytes, stream);
}

int mc_rho2(int32_t N, int32_t M, const mc_tables *t, const double *C_d, double *rho2_d,
            void *ws_d, size_t ws_bytes, mc_stream stream)
{
    if (M > 8) return MC_EINVAL;
    return map_rho(2, N, M, t, C_d, rho2_d, ws_d, ws_bytes, stream);
}

}  // extern "C"
