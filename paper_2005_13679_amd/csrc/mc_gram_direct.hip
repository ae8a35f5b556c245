// Table-free density matrices (Eqs. rho1, rho2): the Gram kernels of
// mc_gram.h over the configurations of N - 1 and N - 2 particles, enumerated
// by index, with the targets in closed form.
#include "mc_gram.h"

namespace mc {
namespace {

int direct_rho(int L, int32_t N, int32_t M, const double *C_d, double *out_d, void *ws_d,
               size_t ws_bytes, mc_stream stream)
{
    int st = check_nm(N, M);
    if (st) return st;
    if (M > 8) return MC_EINVAL;
    const int64_t DN = dim_checked(N, M);
    if (DN < 0 || DN >= ((int64_t)1 << 31)) return MC_ERANGE;
    if (!C_d || !out_d) return MC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (N < L) return gram_zero(M, L, out_d, s);   // no configuration of N - L particles
    const int64_t Dl = dim_checked(N - L, M);
    GramShape gs;
    st = gram_shape(M, L, (Dl + 63) / 64, &gs);
    if (st) return st;
    if (!ws_d) return MC_EINVAL;
    if (ws_bytes < gs.ws) return MC_ENOMEM;
    const bool big = DN * 16 > (int64_t)0xFFFFFFFFu;
    const int Nl = N - L, nbits = bit_width(Nl);
    MC_DISPATCH_M(M, if constexpr (MT > 0 && MT <= 8) {
        if (L == 1) {
            if (big) st = (gram_launch<MT, 1, true>)(DirectSource<MT, 1, true>{Nl, nbits, Dl, DN}, DN, gs, C_d, out_d, ws_d, s);
            else st = (gram_launch<MT, 1, false>)(DirectSource<MT, 1, false>{Nl, nbits, Dl, DN}, DN, gs, C_d, out_d, ws_d, s);
        } else {
            if (big) st = (gram_launch<MT, 2, true>)(DirectSource<MT, 2, true>{Nl, nbits, Dl, DN}, DN, gs, C_d, out_d, ws_d, s);
            else st = (gram_launch<MT, 2, false>)(DirectSource<MT, 2, false>{Nl, nbits, Dl, DN}, DN, gs, C_d, out_d, ws_d, s);
        }
    });
    return st;
}

}  // namespace

size_t gram_workspace(int32_t N, int32_t M, int L)
{
    if (M > 8 || N < L) return 16;
    const int64_t Dl = dim_checked(N - L, M);
    if (Dl < 0) return 0;
    GramShape gs;
    if (gram_shape(M, L, (Dl + 63) / 64, &gs)) return 0;
    return gs.ws;
}

}  // namespace mc

using namespace mc;

extern "C" {

int mc_rho1_direct(int32_t N, int32_t M, const double *C_d, double *rho1_d, void *ws_d,
                   size_t ws_bytes, mc_stream stream)
{
    return direct_rho(1, N, M, C_d, rho1_d, ws_d, ws_bytes, stream);
}

int mc_rho2_direct(int32_t N, int32_t M, const double *C_d, double *rho2_d, void *ws_d,
                   size_t ws_bytes, mc_stream stream)
{
    return direct_rho(2, N, M, C_d, rho2_d, ws_d, ws_bytes, stream);
}

}  // extern "C"
